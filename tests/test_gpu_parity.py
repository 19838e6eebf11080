"""GPU parity: the HIP path through the C-ABI against the CPU oracle.

Bit-exact statistics, tables and pixels; parameters within 1e-4 relative (and
bitwise equal where the binary64 arithmetic is the same, which is expected).
Sizes run from 1x1 frames to the full 14x1920x1080 and uneven rigs, in the
launch configuration the benchmark times."""
import numpy as np
import pytest

from tests.gpu_helpers import (compare_step, gpu_chain_separate, oracle_cams, oracle_opts, rt_cams, say,
                               assert_ints_equal)

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from oracle import ringcorr as rc  # noqa: E402
from paper_1910_03517_amd import rt, synth  # noqa: E402


@pytest.fixture(scope="module", autouse=True)
def need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    rt.load()   # fails loudly if the library is missing


def run_separate(spec_cams, opts, frames_np, pad=0, whole_in_apply=True):
    cams = rt_cams(spec_cams, pad)
    rig = rt.Rig(cams, opts)
    dev = rig.upload(frames_np)
    out = rig.alloc_frames()
    g = gpu_chain_separate(rig, dev, out, whole_in_apply=whole_in_apply)
    for name in ("band_hist", "band_sums", "whole_hist", "whole_sums"):
        assert_ints_equal(g["stats_" + name], g[name], "stats-vs-fused " + name)
    res = compare_step(oracle_cams(cams), oracle_opts(opts), frames_np, g)
    rig.close()
    return res


def test_vga_single_camera_separate_calls():
    say("case: 1x640x480 rgb8, separate calls")
    rig = synth.single_vga()
    frames = synth.rig_frames(rig, 0)
    res = run_separate(rig.cams, rt.Options(), frames)
    assert res["bitwise"], "params not bitwise equal to the binary64 oracle"


SMALL_CASES = [
    # (W, H, C, bit_depth, K, closed, NB, B, pad)
    (1, 1, 3, 8, 1, True, 1, 32, 0),
    (1, 5, 3, 8, 2, True, 4, 32, 1),
    (2, 3, 1, 8, 3, True, 2, 1, 0),
    (3, 7, 3, 8, 2, True, 16, 32, 0),          # H < NB: empty blocks
    (5, 9, 3, 8, 3, False, 4, 2, 2),           # open chain
    (17, 13, 3, 8, 2, True, 3, 32, 1),         # W < 2B: band clamp, ragged groups
    (33, 31, 3, 8, 4, True, 7, 5, 0),
    (64, 48, 1, 8, 2, True, 4, 8, 1),          # gray8
    (61, 40, 1, 10, 2, True, 5, 6, 0),         # 10-bit
    (50, 21, 1, 12, 3, False, 3, 7, 2),        # 12-bit open
    (77, 66, 1, 16, 2, True, 16, 32, 1),       # 16-bit
    (130, 70, 3, 8, 3, True, 16, 32, 0),
    (1031, 67, 3, 8, 2, True, 64, 32, 3),      # several 256-thread passes + tail
]


@pytest.mark.parametrize("case", SMALL_CASES, ids=[f"{c[0]}x{c[1]}x{c[2]}b{c[3]}k{c[4]}" for c in SMALL_CASES])
def test_small_geometries(case):
    W, H, C, bd, K, closed, NB, B, pad = case
    say("case:", case)
    rng = np.random.default_rng(abs(hash(case)) % (2 ** 32))
    spec = [synth.CamSpec(W, H, C, bd, 0, p) for p in range(K)]
    frames = [synth.tiny_frame(H, W, C, bd, rng) for _ in range(K)]
    opts = rt.Options(n_blocks=NB, band_width=B, closed_ring=closed)
    run_separate(spec, opts, frames, pad)


@pytest.mark.parametrize("case", SMALL_CASES, ids=[f"{c[0]}x{c[1]}x{c[2]}b{c[3]}k{c[4]}" for c in SMALL_CASES])
def test_small_geometries_frameset(case):
    """The same geometries through rt_frameset, whose first kernel takes each
    seam block whole (both facing bands, their fits and tables; at the start
    of an open chain also the left band that faces nothing): two frame-sets
    with smoothing, each against the oracle's frame-set sequence."""
    W, H, C, bd, K, closed, NB, B, pad = case
    say("case: frameset", case)
    rng = np.random.default_rng((abs(hash(case)) + 1) % (2 ** 32))
    spec = [synth.CamSpec(W, H, C, bd, 0, p) for p in range(K)]
    cams = rt_cams(spec, pad)
    opts = rt.Options(n_blocks=NB, band_width=B, closed_ring=closed, smoothing=True)
    rig = rt.Rig(cams, opts)
    co, oo = oracle_cams(cams), oracle_opts(opts)
    out = rig.alloc_frames()
    prev_p = prev_v = None
    for t in range(2):
        frames = [synth.tiny_frame(H, W, C, bd, rng) for _ in range(K)]
        dev = rig.upload(frames)
        rig.frameset(dev, out)
        torch.cuda.synchronize()
        g = rig.bufs.host()
        g["out"] = rig.download(out)
        res = compare_step(co, oo, frames, g, prev_p, prev_v)
        assert res["bitwise"], f"frame-set {t}: params not bitwise equal"
        prev_p, prev_v = res["ref"]["params"], res["ref"]["valid"]
    rig.close()


def test_flat_and_saturated_bands():
    """sigma = 0 bands (a = 1 path) and fully saturated cameras."""
    say("case: flat/saturated 3x 96x64")
    rng = np.random.default_rng(7)
    f0 = np.full((64, 96, 3), 255, np.uint8)
    f1 = rng.integers(0, 256, (64, 96, 3)).astype(np.uint8)
    f1[:, :40] = 17
    f2 = np.zeros((64, 96, 3), np.uint8)
    spec = [synth.CamSpec(96, 64, 3, 8, 0, p) for p in range(3)]
    run_separate(spec, rt.Options(n_blocks=4, band_width=16), [f0, f1, f2])


def test_two_rings_mixed_dtypes():
    say("case: two rings rgb8 + u16")
    rng = np.random.default_rng(3)
    spec = ([synth.CamSpec(200, 90, 3, 8, 0, p) for p in (1, 0, 2)]
            + [synth.CamSpec(120, 64, 1, 16, 7, p) for p in (1, 0)])
    frames = [synth.tiny_frame(c.height, c.width, c.channels, c.bit_depth, rng) for c in spec]
    run_separate(spec, rt.Options(n_blocks=8, band_width=12), frames)


def test_inplace_apply():
    say("case: in-place apply 2x 256x40")
    rng = np.random.default_rng(4)
    spec = [synth.CamSpec(256, 40, 3, 8, 0, p) for p in range(2)]
    frames = [synth.tiny_frame(40, 256, 3, 8, rng) for _ in range(2)]
    cams = rt_cams(spec)
    rig = rt.Rig(cams, rt.Options(n_blocks=4))
    dev = rig.upload(frames)
    out = rig.alloc_frames()
    g = gpu_chain_separate(rig, dev, out)
    rig.apply(dev, dev)
    torch.cuda.synchronize()
    for a, b in zip(rig.download(dev), g["out"]):
        assert np.array_equal(a, b)
    rig.close()


def frameset_sequence(rig_spec, opts, n_frames, drift=True, seed=0):
    cams = rt_cams(rig_spec.cams)
    rig = rt.Rig(cams, opts)
    co, oo = oracle_cams(cams), oracle_opts(opts)
    out = rig.alloc_frames()
    prev_p = prev_v = None
    dev = None
    for t in range(n_frames):
        say(f"case: {rig_spec.name} frame {t} smoothing={opts.smoothing}")
        frames = synth.rig_frames(rig_spec, t, drift=drift, seed=seed)
        if dev is None:
            dev = rig.upload(frames)
        else:
            rig.upload_into(dev, frames)
        rig.frameset(dev, out)
        torch.cuda.synchronize()
        g = rig.bufs.host()
        g["out"] = rig.download(out)
        res = compare_step(co, oo, frames, g, prev_p, prev_v)
        assert res["bitwise"], f"frame {t}: params not bitwise equal"
        prev_p, prev_v = res["ref"]["params"], res["ref"]["valid"]
    rig.close()


def test_rig14_frameset_standard():
    frameset_sequence(synth.rig14_1080p(), rt.Options(), 2)


def test_rig14_frameset_smoothing():
    frameset_sequence(synth.rig14_1080p(), rt.Options(smoothing=True), 3)


def pipeline_vs_oracle(spec, n, label, lanes=3, fuse=False):
    """n frame-sets of `spec` (drifting gains, smoothing) through the
    pipeline in one of the bench's launch configurations (8 slots, applies
    issued 3 frame-sets at a time, the last group partial; 3 lanes, or fused:
    a group per launch, 2 lanes): every output against the oracle's
    frame-set sequence, the last two frame-sets' whole-frame statistics and
    the final state bitwise."""
    cams = rt_cams(spec.cams)
    opts = rt.Options(smoothing=True)
    rig = rt.Rig(cams, opts)
    pipe = rt.Pipe.for_rig(rig, depth=8, lanes=lanes, group=3, fuse=fuse)
    frames = [synth.rig_frames(spec, t, drift=True) for t in range(n)]
    dev = [rig.upload(f) for f in frames]
    outs = [rig.alloc_frames() for _ in range(n)]
    torch.cuda.synchronize()
    say(f"case: {label} pipeline, {lanes} lanes, depth 8, group 3, fuse {fuse}, {n} frame-sets")
    slots = [pipe.submit(dev[t], outs[t]) for t in range(n)]
    pipe.join()
    torch.cuda.synchronize()
    rig.check()
    co, oo = oracle_cams(cams), oracle_opts(opts)
    prev_p = prev_v = None
    for t in range(n):
        ref = rc.frameset(co, oo, frames[t], prev_p, prev_v)
        prev_p, prev_v = ref["params"], ref["valid"]
        for k, (x, y) in enumerate(zip(rig.download(outs[t]), ref["out"])):
            assert np.array_equal(x, y), f"frame-set {t} camera {k}"
        if t >= n - 2:
            w = pipe.whole[slots[t]]
            assert np.array_equal(w.whole_hist.cpu().numpy().astype(np.int64), ref["whole_hist"]), f"t {t}"
    h = rig.bufs.host()
    assert np.array_equal(h["params"].view(np.uint64), prev_p.view(np.uint64))
    assert np.array_equal(h["valid"], prev_v)
    pipe.close()
    rig.close()


def test_rig14_lanes_pipeline_matches_oracle():
    """Ten 14x1920x1080 RGB8 frame-sets (two slots reused) through the
    pipeline against the oracle."""
    pipeline_vs_oracle(synth.rig14_1080p(), 10, "rig14")


def test_rig14_fused_pipeline_matches_oracle():
    """The bench's fused form (2 lanes, groups of 3 in one apply launch) on
    ten 14x1920x1080 RGB8 frame-sets against the oracle."""
    pipeline_vs_oracle(synth.rig14_1080p(), 10, "rig14", lanes=2, fuse=True)


def test_uneven_rig_fused_pipeline_matches_oracle():
    """The fused form on five frame-sets of the uneven three-ring rig (16
    cameras, the most a fused launch takes)."""
    pipeline_vs_oracle(synth.uneven_rig(), 5, "uneven rig", lanes=2, fuse=True)


def test_uneven_rig_lanes_pipeline_matches_oracle():
    """Five frame-sets of the uneven three-ring rig (4x4096x2160 RGB8,
    8x1920x1080 RGB8, 4x640x512 gray16) through the pipeline against the
    oracle."""
    pipeline_vs_oracle(synth.uneven_rig(), 5, "uneven rig")


def test_rig14_ahead_loop_matches_oracle():
    """Six drifting 14x1080p frame-sets (smoothing) through rt_frameset_ahead,
    one launch per frame-set: every output, every frame-set's whole-frame
    histogram and the final state against the oracle's sequence, bitwise."""
    spec = synth.rig14_1080p()
    cams = rt_cams(spec.cams)
    opts = rt.Options(smoothing=True)
    rig = rt.Rig(cams, opts)
    n = 6
    frames = [synth.rig_frames(spec, t, drift=True) for t in range(n)]
    dev = [rig.upload(f) for f in frames]
    outs = [rig.alloc_frames() for _ in range(n)]
    luts = [rt.LutSet(rig.sizes) for _ in range(2)]
    wholes = [rt.WholeSet(rig.sizes) for _ in range(2)]
    torch.cuda.synchronize()
    say(f"case: rig14 look-ahead loop, {n} frame-sets")
    co, oo = oracle_cams(cams), oracle_opts(opts)
    prev_p = prev_v = None
    rt.rt_frameset_ahead(rig.ctx, None, None, None, None, dev[0], luts[0], wholes[0], rig.bufs)
    for t in range(n):
        a, e = t % 2, (t + 1) % 2
        nxt = t + 1 < n
        rt.rt_frameset_ahead(rig.ctx, dev[t], outs[t], luts[a], wholes[a], dev[t + 1] if nxt else None,
                             luts[e] if nxt else None, wholes[e] if nxt else None, rig.bufs)
        torch.cuda.synchronize()
        ref = rc.frameset(co, oo, frames[t], prev_p, prev_v)
        prev_p, prev_v = ref["params"], ref["valid"]
        for k, (x, y) in enumerate(zip(rig.download(outs[t]), ref["out"])):
            assert np.array_equal(x, y), f"frame-set {t} camera {k}"
        assert np.array_equal(wholes[a].whole_hist.cpu().numpy().astype(np.int64), ref["whole_hist"]), f"t {t}"
    rig.check()
    h = rig.bufs.host()
    assert np.array_equal(h["params"].view(np.uint64), prev_p.view(np.uint64))
    assert np.array_equal(h["valid"], prev_v)
    rig.close()


def test_uneven_rig_frameset():
    frameset_sequence(synth.uneven_rig(), rt.Options(), 1)


def test_determinism_repeated_runs():
    """Integer atomics are order independent: 20 runs must agree bit for bit."""
    say("case: determinism 14x1920x1080 x20")
    spec = synth.rig14_1080p()
    cams = rt_cams(spec.cams)
    rig = rt.Rig(cams, rt.Options())
    frames = synth.rig_frames(spec, 0)
    dev = rig.upload(frames)
    out = rig.alloc_frames()
    first = None
    for i in range(20):
        rig.bufs.valid.zero_()
        rig.frameset(dev, out)
        torch.cuda.synchronize()
        h = rig.bufs.host()
        cur = (h["band_hist"].tobytes(), h["whole_hist"].tobytes(), h["whole_sums"].tobytes(),
               h["params"].tobytes(), b"".join(o[:, :cams[0].row_bytes].cpu().numpy().tobytes() for o in out))
        if first is None:
            first = cur
        else:
            assert cur == first, f"run {i} differs"
    rig.close()


@pytest.mark.parametrize("tile_rows,grid", [(1, 0), (3, 1), (16, 7), (64, 0), (4096, 2), (2, 5000), (5, 3)])
def test_frameset_tuning_knobs_do_not_change_results(tile_rows, grid):
    """Segment height and apply grid are performance knobs only: one
    workgroup over every row of every camera (the histogram of each camera
    carried across its segments, 8-bit and 12-bit cameras in one run), shares
    that cross cameras, and more workgroups than rows (empty shares)."""
    say(f"case: knobs tile_rows={tile_rows} grid={grid}")
    rng = np.random.default_rng(tile_rows * 31 + grid)
    spec = ([synth.CamSpec(300, 77, 3, 8, 0, p) for p in range(3)]
            + [synth.CamSpec(96, 40, 1, 12, 1, p) for p in range(2)])
    frames = [synth.tiny_frame(c.height, c.width, c.channels, c.bit_depth, rng) for c in spec]
    cams = rt_cams(spec)
    opts = rt.Options(n_blocks=5, band_width=9, smoothing=True)
    rig = rt.Rig(cams, opts)
    rig.tune(tile_rows, grid)
    dev = rig.upload(frames)
    out = rig.alloc_frames()
    prev_p = prev_v = None
    for t in range(2):
        rig.frameset(dev, out)
        rig.check()
        g = rig.bufs.host()
        g["out"] = rig.download(out)
        res = compare_step(oracle_cams(cams), oracle_opts(opts), frames, g, prev_p, prev_v)
        prev_p, prev_v = res["ref"]["params"], res["ref"]["valid"]
    rig.close()


@pytest.mark.parametrize("grid", [1, 2, 3, 7])
def test_knobs_with_empty_blocks(grid):
    """Shares over cameras shorter than the block count (H < NB: some blocks
    hold no rows, so several block starts fall on one row and a share's row
    loop must step over every empty block); 8-bit RGB and gray cameras."""
    say(f"case: empty blocks, grid={grid}")
    rng = np.random.default_rng(100 + grid)
    spec = ([synth.CamSpec(40, 7, 3, 8, 0, p) for p in range(3)]
            + [synth.CamSpec(24, 5, 1, 8, 1, p) for p in range(2)])
    frames = [synth.tiny_frame(c.height, c.width, c.channels, c.bit_depth, rng) for c in spec]
    cams = rt_cams(spec)
    opts = rt.Options(n_blocks=16, band_width=6)
    rig = rt.Rig(cams, opts)
    rig.tune(32, grid)
    dev = rig.upload(frames)
    out = rig.alloc_frames()
    rig.frameset(dev, out)
    rig.check()
    g = rig.bufs.host()
    g["out"] = rig.download(out)
    res = compare_step(oracle_cams(cams), oracle_opts(opts), frames, g)
    assert res["bitwise"]
    rig.close()


@pytest.mark.skip(reason="the single-launch persistent frame-set kernel (in-kernel dependency waits) did not "
                         "complete on its first two device runs; it is switched off (not built) until its cause "
                         "is shown, and rt_frameset uses the four-kernel sequence")
def test_persistent_single_launch_frameset():
    frameset_sequence(synth.rig14_1080p(), rt.Options(), 1)


@pytest.mark.parametrize("vec", [4, 8, 12, 16])
def test_stream_copy_utility(vec):
    say(f"case: stream copy vec={vec}")
    n = 1_000_003
    src = torch.randint(0, 256, (n,), dtype=torch.uint8, device="cuda")
    dst = torch.zeros(n, dtype=torch.uint8, device="cuda")
    rt.rt_stream_copy(dst, src, n, vec)
    torch.cuda.synchronize()
    assert torch.equal(src, dst)


@pytest.mark.parametrize("depth,lanes,group", [(1, 1, 1), (2, 1, 1), (3, 1, 1), (2, 2, 1), (3, 2, 1), (4, 3, 1),
                                               (4, 4, 1), (4, 2, 2), (3, 1, 3), (5, 3, 3), (8, 2, 4)])
def test_pipeline_matches_sequential_framesets(depth, lanes, group):
    """Pipelining of consecutive frame-sets (statistics and estimates on one
    stream, applies round-robin over `lanes` streams and issued `group` at a
    time, `depth` slots reused over 11 frame-sets, the last group partial)
    gives the results of consecutive rt_frameset calls, bit for bit
    (smoothing mode, drifting gains)."""
    say(f"case: pipeline depth {depth} lanes {lanes} group {group} vs sequential, 4x 480x200 rgb8, 11 frame-sets")
    spec = synth.RigSpec("pipe 4x480x200", 11, [synth.CamSpec(480, 200, 3, 8, 0, p) for p in range(4)])
    cams = rt_cams(spec.cams)
    opts = rt.Options(n_blocks=8, band_width=16, smoothing=True)
    seq = rt.Rig(cams, opts)
    par = rt.Rig(cams, opts)
    pipe = rt.Pipe.for_rig(par, depth=depth, lanes=lanes, group=group)
    T = 11
    frames_t = [synth.rig_frames(spec, t, drift=True) for t in range(T)]
    dev = [seq.upload(f) for f in frames_t]
    torch.cuda.synchronize()
    outs_p = [par.alloc_frames() for _ in range(T)]
    slots = [pipe.submit(dev[t], outs_p[t]) for t in range(T)]
    pipe.join()
    torch.cuda.synchronize()
    out_s = seq.alloc_frames()
    for t in range(T):
        seq.frameset(dev[t], out_s)
        torch.cuda.synchronize()
        hs = seq.bufs.host()
        if t >= T - depth:   # slots of the last `depth` frame-sets are still intact
            w = pipe.whole[slots[t]]
            assert np.array_equal(w.whole_hist.cpu().numpy(), seq.bufs.whole_hist.cpu().numpy())
            assert np.array_equal(w.whole_sums.cpu().numpy(), seq.bufs.whole_sums.cpu().numpy())
            L = pipe.luts[slots[t]]
            assert np.array_equal(L.lut8.cpu().numpy(), seq.bufs.lut8.cpu().numpy())
        for a, b in zip(par.download(outs_p[t]), seq.download(out_s)):
            assert np.array_equal(a, b), f"frame-set {t}"
    hp = par.bufs.host()
    assert np.array_equal(hp["params"].view(np.uint64), hs["params"].view(np.uint64))
    pipe.close()
    seq.close()
    par.close()


def test_pipeline_caller_stream_changes():
    """Submits that switch between two caller streams inside groups of 3
    (3 lanes, 6 slots, 8 frame-sets): a stream change issues the pending
    applies on their own stream first, and the outputs and final state equal
    consecutive rt_frameset calls bit for bit."""
    say("case: pipeline 3 lanes, depth 6, group 3, caller stream alternating, 4x 480x200 rgb8, 8 frame-sets")
    spec = synth.RigSpec("pipe streams 4x480x200", 12, [synth.CamSpec(480, 200, 3, 8, 0, p) for p in range(4)])
    cams = rt_cams(spec.cams)
    opts = rt.Options(n_blocks=8, band_width=16, smoothing=True)
    seq = rt.Rig(cams, opts)
    par = rt.Rig(cams, opts)
    pipe = rt.Pipe.for_rig(par, depth=6, lanes=3, group=3)
    T = 8
    dev = [seq.upload(synth.rig_frames(spec, t, drift=True)) for t in range(T)]
    outs_p = [par.alloc_frames() for _ in range(T)]
    torch.cuda.synchronize()
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    for t in range(T):
        pipe.submit(dev[t], outs_p[t], stream=streams[(t // 2) % 2])
    for s in streams:
        pipe.join(s)
    torch.cuda.synchronize()
    out_s = seq.alloc_frames()
    for t in range(T):
        seq.frameset(dev[t], out_s)
        torch.cuda.synchronize()
        for a, b in zip(par.download(outs_p[t]), seq.download(out_s)):
            assert np.array_equal(a, b), f"frame-set {t}"
    hp, hs = par.bufs.host(), seq.bufs.host()
    assert np.array_equal(hp["params"].view(np.uint64), hs["params"].view(np.uint64))
    pipe.close()
    seq.close()
    par.close()


def test_pipeline_mixed_rings_matches_sequential():
    """Mixed rings through the pipeline (3 lanes, groups of 3): a closed RGB8
    ring, an open gray16 chain and a one-camera RGB8 ring, 7 frame-sets with
    smoothing; every output and the final state equal consecutive rt_frameset
    calls, and the last frame-sets' whole-frame statistics and tables equal
    theirs."""
    say("case: pipeline mixed rings, 3 lanes, depth 6, group 3, 7 frame-sets")
    cams_spec = ([synth.CamSpec(200, 90, 3, 8, 0, p) for p in (1, 0, 2)]
                 + [synth.CamSpec(120, 64, 1, 16, 4, p) for p in (1, 0)]
                 + [synth.CamSpec(160, 48, 3, 8, 9, 0)])
    cams = rt_cams(cams_spec, 1)
    opts = rt.Options(n_blocks=5, band_width=12, smoothing=True, closed_ring=False)
    seq = rt.Rig(cams, opts)
    par = rt.Rig(cams, opts)
    depth = 6
    pipe = rt.Pipe.for_rig(par, depth=depth, lanes=3, group=3)
    rng = np.random.default_rng(21)
    T = 7
    frames_t = [[synth.tiny_frame(c.height, c.width, c.channels, c.bit_depth, rng) for c in cams_spec]
                for _ in range(T)]
    dev = [seq.upload(f) for f in frames_t]
    outs_p = [par.alloc_frames() for _ in range(T)]
    torch.cuda.synchronize()
    slots = [pipe.submit(dev[t], outs_p[t]) for t in range(T)]
    pipe.join()
    torch.cuda.synchronize()
    out_s = seq.alloc_frames()
    for t in range(T):
        seq.frameset(dev[t], out_s)
        torch.cuda.synchronize()
        if t >= T - depth:
            w = pipe.whole[slots[t]]
            assert np.array_equal(w.whole_hist.cpu().numpy(), seq.bufs.whole_hist.cpu().numpy()), f"t {t}"
            assert np.array_equal(w.whole_sums.cpu().numpy(), seq.bufs.whole_sums.cpu().numpy()), f"t {t}"
            L = pipe.luts[slots[t]]
            assert np.array_equal(L.q16.cpu().numpy(), seq.bufs.q16.cpu().numpy()), f"t {t}"
        for k, (a, b) in enumerate(zip(par.download(outs_p[t]), seq.download(out_s))):
            assert np.array_equal(a, b), f"frame-set {t} camera {k}"
    hp, hs = par.bufs.host(), seq.bufs.host()
    assert np.array_equal(hp["params"].view(np.uint64), hs["params"].view(np.uint64))
    assert np.array_equal(hp["valid"], hs["valid"])
    pipe.close()
    seq.close()
    par.close()


def test_pipeline_waits_for_ready_event():
    """Frames written on a side stream right before each submit, ordered
    only by the ready event the submit passes: the results equal consecutive
    rt_frameset calls on the same frames."""
    say("case: pipeline ready_event, 3 lanes, 4x 480x200 rgb8, 7 frame-sets")
    spec = synth.RigSpec("pipe 4x480x200", 13, [synth.CamSpec(480, 200, 3, 8, 0, p) for p in range(4)])
    cams = rt_cams(spec.cams)
    opts = rt.Options(n_blocks=8, band_width=16, smoothing=True)
    seq = rt.Rig(cams, opts)
    par = rt.Rig(cams, opts)
    pipe = rt.Pipe.for_rig(par, depth=6, lanes=3, group=3)
    T = 7
    frames_t = [synth.rig_frames(spec, t, drift=True) for t in range(T)]
    src = [seq.upload(f) for f in frames_t]          # device copies, written once
    torch.cuda.synchronize()
    dst = [par.alloc_frames() for _ in range(T)]     # written on the side stream below
    outs = [par.alloc_frames() for _ in range(T)]
    torch.cuda.synchronize()
    side = torch.cuda.Stream()
    for t in range(T):
        with torch.cuda.stream(side):
            for a, b in zip(dst[t], src[t]):
                a.copy_(b, non_blocking=True)
        ready = torch.cuda.Event()
        ready.record(side)
        pipe.submit(dst[t], outs[t], ready_event=ready)
    pipe.join()
    torch.cuda.synchronize()
    out_s = seq.alloc_frames()
    for t in range(T):
        seq.frameset(src[t], out_s)
        torch.cuda.synchronize()
        for a, b in zip(par.download(outs[t]), seq.download(out_s)):
            assert np.array_equal(a, b), f"frame-set {t}"
    pipe.close()
    seq.close()
    par.close()


def test_pipeline_rejects_bad_lanes_and_groups():
    spec = synth.RigSpec("pipe 2x64x32", 12, [synth.CamSpec(64, 32, 3, 8, 0, p) for p in range(2)])
    rig = rt.Rig(rt_cams(spec.cams), rt.Options(n_blocks=2, band_width=8))
    for depth, lanes, group, needle in [(2, 0, 1, "lanes"), (4, 5, 1, "lanes"), (2, 3, 1, "below"),
                                        (2, 1, 0, "group"), (2, 1, 3, "group")]:
        luts = [rt.LutSet(rig.sizes) for _ in range(depth)]
        wholes = [rt.WholeSet(rig.sizes) for _ in range(depth)]
        with pytest.raises(rt.RtError, match=needle):
            rt.Pipe(rig.ctx, rig.bufs, luts, wholes, lanes=lanes, group=group)
    rig.close()


def _eager_sequence(cams, opts, dev_frames, order):
    """Consecutive rt_frameset calls; per step copies of out, whole stats, params."""
    rig = rt.Rig(cams, opts)
    out = rig.alloc_frames()
    res = []
    for i in order:
        rig.frameset(dev_frames[i], out)
        torch.cuda.synchronize()
        res.append(dict(out=rig.download(out), wh=rig.bufs.whole_hist.cpu().numpy().copy(),
                        ws=rig.bufs.whole_sums.cpu().numpy().copy(), params=rig.bufs.params.cpu().numpy().copy()))
    rig.close()
    return res


@pytest.mark.parametrize("pipelined", [False, True])
def test_graph_replays_match_eager(pipelined):
    """Captured frame-set graphs, replayed over a cycle of 4 input buffers for 8
    steps with eager torch work and synchronizations between replays: every
    replay equals the eager rt_frameset result of the same step."""
    say(f"case: graph replay pipelined={pipelined}, 3x352x144 rgb8 + 2x96x64 u12")
    spec = synth.RigSpec("graph", 12, [synth.CamSpec(352, 144, 3, 8, 0, p) for p in range(3)]
                         + [synth.CamSpec(96, 64, 1, 12, 1, p) for p in range(2)])
    cams = rt_cams(spec.cams)
    opts = rt.Options(n_blocks=6, band_width=12, smoothing=True)
    rig = rt.Rig(cams, opts)
    frames = [synth.rig_frames(spec, t, drift=True) for t in range(4)]
    dev = [rig.upload(f) for f in frames]
    torch.cuda.synchronize()
    order = [t % 4 for t in range(8)]
    eager = _eager_sequence(cams, opts, dev, order)
    luts = [rt.LutSet(rig.sizes) for _ in range(2)]
    whole = rt.WholeSet(rig.sizes)
    out = rig.alloc_frames()
    b = rig.bufs
    if pipelined:
        rt.rt_stats(rig.ctx, dev[0], b.band_hist, b.band_sums)
        rt.rt_estimate(rig.ctx, b.band_hist, b.band_sums, b.params, b.valid)
        rt.rt_build_lut(rig.ctx, b.params, b.valid, luts[0].lut8, luts[0].q16, luts[0].weights)
        graphs = [rt.Graph(rig.ctx, dev[i], out, luts[i % 2], whole, b, dev[(i + 1) % 4], luts[(i + 1) % 2])
                  for i in range(4)]
    else:
        graphs = [rt.Graph(rig.ctx, dev[i], out, luts[0], whole, b) for i in range(4)]
    scratch = torch.zeros(1 << 20, device="cuda")
    for t, i in enumerate(order):
        graphs[i].launch()
        torch.cuda.synchronize()
        scratch.add_(1.0)                       # eager work between replays
        torch.cuda.synchronize()
        got = rig.download(out)
        for k, (a, e) in enumerate(zip(got, eager[t]["out"])):
            assert np.array_equal(a, e), f"step {t} camera {k}"
        assert np.array_equal(whole.whole_hist.cpu().numpy(), eager[t]["wh"]), f"step {t} whole_hist"
        assert np.array_equal(whole.whole_sums.cpu().numpy(), eager[t]["ws"]), f"step {t} whole_sums"
        if not pipelined:
            assert np.array_equal(b.params.cpu().numpy(), eager[t]["params"]), f"step {t} params"
    rig.check()
    for g in graphs:
        g.close()
    rig.close()


@pytest.mark.parametrize("pipelined,extra", [(False, {}), (True, {}), (False, {"vblend": True, "fit": "quantile"})])
def test_graph_rebound_frames_match_eager(pipelined, extra):
    """One captured graph (two for the two-branch form, which alternate the
    table buffers) serves every input and output buffer: rt_graph_set_frames
    before each launch, over a cycle of 4 inputs and 2 outputs for 9 steps
    with eager torch work between the launches; every launch equals the
    eager rt_frameset result of the same step.  A mismatched next_frames is
    refused."""
    say(f"case: graph set_frames pipelined={pipelined} {extra}, 3x352x144 rgb8 + 2x96x64 u12")
    spec = synth.RigSpec("graph rebind", 14, [synth.CamSpec(352, 144, 3, 8, 0, p) for p in range(3)]
                         + [synth.CamSpec(96, 64, 1, 12, 1, p) for p in range(2)])
    cams = rt_cams(spec.cams)
    opts = rt.Options(n_blocks=6, band_width=12, smoothing=True, **extra)
    rig = rt.Rig(cams, opts)
    frames = [synth.rig_frames(spec, t, drift=True) for t in range(4)]
    dev = [rig.upload(f) for f in frames]
    torch.cuda.synchronize()
    order = [(3 * t) % 4 for t in range(9)]
    eager = _eager_sequence(cams, opts, dev, order)
    luts = [rt.LutSet(rig.sizes) for _ in range(2)]
    whole = rt.WholeSet(rig.sizes)
    outs = [rig.alloc_frames() for _ in range(2)]
    b = rig.bufs
    if pipelined:
        rt.rt_stats(rig.ctx, dev[order[0]], b.band_hist, b.band_sums)
        rt.rt_estimate(rig.ctx, b.band_hist, b.band_sums, b.params, b.valid)
        rt.rt_build_lut(rig.ctx, b.params, b.valid, luts[0].lut8, luts[0].q16, luts[0].weights)
        # captured on buffers of no step, so that every launch is rebound
        graphs = [rt.Graph(rig.ctx, dev[1], outs[1], luts[p], whole, b, dev[2], luts[1 - p]) for p in range(2)]
        with pytest.raises(rt.RtError, match="next_frames"):
            graphs[0].set_frames(dev[0], outs[0])
    else:
        graphs = [rt.Graph(rig.ctx, dev[1], outs[1], luts[0], whole, b)]
        with pytest.raises(rt.RtError, match="next_frames"):
            graphs[0].set_frames(dev[0], outs[0], dev[1])
    scratch = torch.zeros(1 << 20, device="cuda")
    for t, i in enumerate(order):
        g = graphs[t % len(graphs)]
        out = outs[t % 2]
        if pipelined:
            g.set_frames(dev[i], out, dev[order[(t + 1) % len(order)]])
        else:
            g.set_frames(dev[i], out)
        g.launch()
        torch.cuda.synchronize()
        scratch.add_(1.0)                       # eager work between launches
        torch.cuda.synchronize()
        got = rig.download(out)
        for k, (a, e) in enumerate(zip(got, eager[t]["out"])):
            assert np.array_equal(a, e), f"step {t} camera {k}"
        assert np.array_equal(whole.whole_hist.cpu().numpy(), eager[t]["wh"]), f"step {t} whole_hist"
        if not pipelined:
            assert np.array_equal(b.params.cpu().numpy(), eager[t]["params"]), f"step {t} params"
    if not pipelined:
        # Rebinds between launches that are still queued or running: each
        # launch keeps the frames it was launched with.
        more = [(3 * t + 1) % 4 for t in range(6)]
        eager2 = _eager_sequence(cams, opts, dev, order + more)[len(order):]
        outs2 = [rig.alloc_frames() for _ in more]
        torch.cuda.synchronize()
        g = graphs[0]
        for t, i in enumerate(more):
            g.set_frames(dev[i], outs2[t])
            g.launch()
        torch.cuda.synchronize()
        for t in range(len(more)):
            for k, (a, e) in enumerate(zip(rig.download(outs2[t]), eager2[t]["out"])):
                assert np.array_equal(a, e), f"queued step {t} camera {k}"
        assert np.array_equal(b.params.cpu().numpy(), eager2[-1]["params"])
    rig.check()
    for g in graphs:
        g.close()
    rig.close()


@pytest.mark.parametrize("channels,bit_depth", [(3, 8), (1, 16)])
def test_whole_histogram_counters_do_not_overflow(channels, bit_depth):
    """A flat 8192-wide frame puts every sample of a tile into one bin; with
    tile_rows 4096 no counter of the apply pass's histogram may wrap (with the
    packed 16-bit layout the tile builder splits the 300-row block)."""
    say(f"case: flat 8192x300 c{channels} b{bit_depth}, tile_rows 4096")
    W, H = 8192, 300
    spec = [synth.CamSpec(W, H, channels, bit_depth, 0, 0)]
    cams = rt_cams(spec)
    opts = rt.Options(n_blocks=1)
    rig = rt.Rig(cams, opts)
    rig.tune(4096, 0)
    dt = np.uint8 if bit_depth == 8 else np.uint16
    frame = np.full((H, W, channels), 200 if bit_depth == 8 else 51234, dt)
    dev = rig.upload([frame])
    out = rig.alloc_frames()
    g = gpu_chain_separate(rig, dev, out)
    compare_step(oracle_cams(cams), oracle_opts(opts), [frame], g)
    rig.close()


def test_huge_gains_use_the_tables():
    """Gains whose Q16 slope needs more than 24 bits (a up to a_max = 1000)
    cannot be evaluated directly in 32-bit integers; those tiles must take the
    table path and still match the oracle bit for bit."""
    say("case: huge gains, a_max 1000")
    rng = np.random.default_rng(77)
    W, H = 128, 64
    spec = [synth.CamSpec(W, H, 3, 8, 0, p) for p in range(2)]
    f0 = np.full((H, W, 3), 100, np.uint8)
    f0[::7, ::5, :] = 101                          # nearly flat: tiny but non-zero spread
    f1 = rng.integers(0, 256, (H, W, 3)).astype(np.uint8)
    cams = rt_cams(spec)
    opts = rt.Options(n_blocks=2, band_width=16, a_max=1000.0)
    rig = rt.Rig(cams, opts)
    dev = rig.upload([f0, f1])
    out = rig.alloc_frames()
    g = gpu_chain_separate(rig, dev, out)
    assert np.abs(g["q16"][..., 0]).max() >= (1 << 23), "the case must exceed the direct range"
    compare_step(oracle_cams(cams), oracle_opts(opts), [f0, f1], g)
    rig.frameset(dev, out)
    rig.check()
    rig.close()
