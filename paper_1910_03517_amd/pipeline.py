"""Frame-set pipeline over the C-ABI (rt_pipe).

Per frame-set the same kernels as rt_frameset run, split over two HIP
streams by the library: the band statistics, estimate and tables of
frame-set t+1 run on the pipeline's own stream while the bandwidth-bound
apply of frame-set t runs on the caller's stream.  Tables and whole-frame
statistics rotate over `depth` slots; band statistics and the estimator
state are single buffers, so the results are exactly those of consecutive
rt_frameset calls.  This module only allocates the slot buffers and
marshals arguments.
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
    """Overlaps the estimate of frame-set t+1 with the apply of frame-set t.

    alternate=True: whole frame-sets alternate between the caller's stream and
    the pipeline's own (rt_pipe_create_alternating); call join() before
    depending on the caller's stream for all submitted work."""

    def __init__(self, rig: rt.Rig, depth: int = 2, alternate: bool = False):
        self.rig = rig
        self.depth = 2 if alternate else depth
        self.luts = [LutSet(rig.sizes, rig.device) for _ in range(self.depth)]
        self.whole = [WholeSet(rig.sizes, rig.device) for _ in range(self.depth)]
        self.pipe = rt.Pipe(rig.ctx, rig.bufs, self.luts, self.whole, alternate=alternate)

    def submit(self, frames, out_frames, stream=None, frame_ptrs=None, out_ptrs=None, ready_event=None) -> int:
        """Enqueue one frame-set on `stream` (default: torch's current stream); returns its slot.

        The frames must be written before the statistics read them: pass
        ready_event (recorded after the write) unless they were written and
        synchronized earlier."""
        return self.pipe.submit(frames, out_frames, stream, frame_ptrs, out_ptrs, ready_event)

    def join(self, stream=None) -> None:
        self.pipe.join(stream)

    def close(self) -> None:
        self.pipe.close()
