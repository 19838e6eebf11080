"""Frame-set pipeline over the C-ABI (rt_pipe).

Per frame-set the same kernels as rt_frameset run, split over HIP streams by
the library: the band statistics, estimate and tables of each frame-set run
in order on the pipeline's own stream, ahead of the bandwidth-bound applies,
which go round-robin over one or more lanes (the caller's stream, then
streams of the pipeline).  Tables and whole-frame statistics rotate over
`depth` slots; band statistics and the estimator state are single buffers,
so the results are exactly those of consecutive rt_frameset calls.  This
module only allocates the slot buffers and marshals arguments.
"""
from __future__ import annotations

from . import rt


class LutSet:
    def __init__(self, sizes: rt.rt_sizes, device="cuda"):
        import torch
        K, NB, WM = sizes.n_cams, sizes.n_blocks, max(sizes.w_max, 1)
        self.lut8 = torch.zeros((K, 2, NB, rt.CSLOTS, rt.NBINS), dtype=torch.uint8, device=device)
        self.q16 = torch.zeros((K, 2, NB, rt.CSLOTS, 2), dtype=torch.int64, device=device)
        self.weights = torch.zeros((K, WM), dtype=torch.int16, device=device)


class WholeSet:
    def __init__(self, sizes: rt.rt_sizes, device="cuda"):
        import torch
        K = sizes.n_cams
        self.whole_hist = torch.zeros((K, rt.CSLOTS, rt.NBINS), dtype=torch.int32, device=device)
        self.whole_sums = torch.zeros((K, rt.CSLOTS, 3), dtype=torch.int64, device=device)


class Pipeline:
    """Band statistics and estimates of consecutive frame-sets run in order on
    the pipeline's stream while the applies go round-robin over `lanes`
    streams (the caller's first), so the estimate of frame-set t+1 overlaps
    the apply of frame-set t, and with lanes > 1 the applies of consecutive
    frame-sets overlap each other.  Applies are issued `group` frame-sets at
    a time (one cross-stream dependency per lane and group).  `depth` slots
    of tables and whole-frame statistics (>= lanes, >= group; 2 * group lets
    the estimates run a group ahead).  Call join() before depending on the
    results of submitted frame-sets."""

    def __init__(self, rig: rt.Rig, depth: int = 2, lanes: int = 1, group: int = 1):
        self.rig = rig
        self.depth = depth
        self.lanes = lanes
        self.group = group
        self.luts = [LutSet(rig.sizes, rig.device) for _ in range(self.depth)]
        self.whole = [WholeSet(rig.sizes, rig.device) for _ in range(self.depth)]
        self.pipe = rt.Pipe(rig.ctx, rig.bufs, self.luts, self.whole, lanes=lanes, group=group)

    def submit(self, frames, out_frames, stream=None, frame_ptrs=None, out_ptrs=None, ready_event=None) -> int:
        """Enqueue one frame-set on `stream` (default: torch's current stream); returns its slot.

        The frames must be written before the statistics read them: pass
        ready_event (recorded after the write) unless they were written and
        synchronized earlier."""
        return self.pipe.submit(frames, out_frames, stream, frame_ptrs, out_ptrs, ready_event)

    def submit_batch(self, active: int, frames, out_frames, stream=None, ready_event=None, done_event=None) -> int:
        """submit() for the cameras in bitmask `active` (whole rings); see rt_pipe_submit_batch."""
        return self.pipe.submit_batch(active, frames, out_frames, stream, ready_event, done_event)

    def join(self, stream=None) -> None:
        self.pipe.join(stream)

    def close(self) -> None:
        self.pipe.close()
