"""The server on the device: three rigs in one context, continuously batched.
Each rig's outputs in the mix equal the oracle's frame-set sequence of that
rig (bit for bit), and equal the rig served alone; with the surrogate
(forced to be used wherever eligible) the mix equals the rig alone."""
import numpy as np
import pytest

from tests.gpu_helpers import oracle_cams, oracle_opts, rt_cams, say

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from oracle import ringcorr as rc  # noqa: E402
from paper_1910_03517_amd import rt, synth  # noqa: E402
from paper_1910_03517_amd.serving import GpuBackend, Server, ShardedBackend  # noqa: E402
from paper_1910_03517_amd.surrogate import Surrogate, Workspace  # noqa: E402


@pytest.fixture(scope="module", autouse=True)
def need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    rt.load()


RIGS = [synth.ring_of(3, 320, 96), synth.ring_of(2, 256, 64), synth.ring_of(4, 200, 48)]
OPTS = rt.Options(n_blocks=4, band_width=16, smoothing=True)
N_PER_RIG = [5, 3, 4]


def rig_frames(r, t):
    spec = synth.RigSpec(f"serving rig {r}", 40 + r, RIGS[r])
    return synth.rig_frames(spec, t, drift=True)


def to_device(cams, frames):
    out = []
    for c, f in zip(cams, frames):
        d = torch.zeros((c.height, c.pitch_bytes), dtype=torch.uint8, device="cuda")
        raw = np.ascontiguousarray(f).view(np.uint8).reshape(c.height, c.row_bytes)
        d[:, :c.row_bytes].copy_(torch.from_numpy(raw))
        out.append(d)
    return out


def host_out(cams, outs):
    res = []
    for d, c in zip(outs, cams):
        raw = d[:, :c.row_bytes].cpu().numpy()
        res.append(np.ascontiguousarray(raw).reshape(c.height, c.width, c.channels))
    return res


def serve(surrogate=None, lanes=1, producer=False, max_cams=None):
    """Every frame-set of every rig through the server.  producer: the input
    frames start out zero and are written by a separate producer stream (a
    stand-in for a decoder) behind some delaying work; each request carries
    the event recorded after its write, and the server's device work must
    wait for it."""
    if max_cams is None:
        backend = GpuBackend(RIGS, OPTS, surrogate=surrogate, lanes=lanes)
    else:
        backend = ShardedBackend(RIGS, OPTS, max_cams=max_cams, surrogate=surrogate, lanes=lanes)
    results = {}

    def on_done(req):
        cams = backend.rig_cams(req.rig)
        results[(req.rig, req.seq)] = host_out(cams, req.out)

    srv = Server(backend, mem_budget=max(N_PER_RIG) * sum(backend.frameset_bytes(r) for r in range(3)),
                 max_batches_in_flight=2, on_done=on_done)
    inputs = {}
    order = [(r, t) for t in range(max(N_PER_RIG)) for r in range(3) if t < N_PER_RIG[r]]
    staged = {}
    for r, t in order:
        cams = backend.rig_cams(r)
        inputs[(r, t)] = to_device(cams, rig_frames(r, t))
        if producer:
            staged[(r, t)] = inputs[(r, t)]
            inputs[(r, t)] = [torch.zeros_like(d) for d in staged[(r, t)]]
    torch.cuda.synchronize()                     # the backend's streams do not wait for this one
    ready = {}
    if producer:
        ps = torch.cuda.Stream()
        busy = torch.rand((2048, 2048), device="cuda")
        with torch.cuda.stream(ps):
            for r, t in order:
                for _ in range(4):
                    busy = busy @ busy
                    busy = busy / busy.abs().amax()
                for d, src in zip(inputs[(r, t)], staged[(r, t)]):
                    d.copy_(src)
                ev = torch.cuda.Event()
                ev.record(ps)
                ready[(r, t)] = ev
    # Everything arrives before the first scheduling pass, so launches carry
    # one frame-set of every rig that still has one (batches of 3, 3, 3, 2, 1).
    for r, t in order:
        req = srv.submit(r, inputs[(r, t)], ready=ready.get((r, t)))
        assert req.seq == t
    srv.drain(timeout=60)
    rep = srv.report()
    say(f"serving report: {rep}")
    assert rep["done"] == sum(N_PER_RIG), rep
    assert sorted(srv.batch_sizes, reverse=True) == [3, 3, 3, 2, 1], srv.batch_sizes
    backend.close()
    return results


@pytest.mark.parametrize("lanes,producer,max_cams", [(1, False, None), (2, False, None), (1, True, None),
                                                     (2, True, None), (1, False, 5), (2, True, 4)])
def test_serving_mix_matches_oracle_and_alone(lanes, producer, max_cams):
    """lanes 1: one rt_frameset_batch per batch on one stream; lanes 2: the
    batches through the frame-set pipeline, consecutive ones overlapping.
    producer: the frames are written by another stream, ordered by the
    requests' ready events.  max_cams: the rigs spread over several contexts
    (ShardedBackend; 5 cameras: two contexts, 4: three), each batch split
    into one launch per context."""
    say(f"case: serving plain, 3 rigs, {lanes} lanes, producer stream {producer}, max_cams {max_cams}")
    results = serve(lanes=lanes, producer=producer, max_cams=max_cams)
    for r in range(3):
        cams = rt_cams(RIGS[r])
        co, oo = oracle_cams(cams), oracle_opts(OPTS)
        prev_p = prev_v = None
        alone = rt.Rig(cams, OPTS)
        for t in range(N_PER_RIG[r]):
            fr = rig_frames(r, t)
            ref = rc.frameset(co, oo, fr, prev_p, prev_v)
            prev_p, prev_v = ref["params"], ref["valid"]
            dev = alone.upload(fr)
            out = alone.alloc_frames()
            alone.frameset(dev, out)
            got_alone = alone.download(out)
            for k in range(len(cams)):
                assert np.array_equal(results[(r, t)][k], ref["out"][k]), f"rig {r} t {t} cam {k} vs oracle"
                assert np.array_equal(results[(r, t)][k], got_alone[k]), f"rig {r} t {t} cam {k} vs alone"
        alone.close()


def test_serving_surrogate_mix_matches_alone():
    say("case: serving surrogate, 3 rigs")
    w = rt.MlpTensors(synth.mlp_init(3))
    sur = Surrogate(w, tol=1e30)          # use the network wherever a unit is eligible
    results = serve(sur)
    for r in range(3):
        cams = rt_cams(RIGS[r])
        alone = rt.Rig(cams, OPTS)
        ws = Workspace(alone.sizes)
        for t in range(N_PER_RIG[r]):
            dev = alone.upload(rig_frames(r, t))
            out = alone.alloc_frames()
            sur.frameset(alone, dev, out, alone.bufs.whole_hist, ws)
            got = alone.download(out)
            for k in range(len(cams)):
                assert np.array_equal(results[(r, t)][k], got[k]), f"rig {r} t {t} cam {k}"
        alone.close()
