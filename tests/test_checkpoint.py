"""Trainer checkpoints: save / load round-trips every tensor, the step count,
the learning rate and the mini-batch permutation generator bit for bit (CPU
tensors), refuses a mismatched batch size, and holds nothing that needs
unpickling."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_1910_03517_amd import rt, synth  # noqa: E402
from paper_1910_03517_amd import surrogate as su  # noqa: E402


def _trainer(seed=3, batch=128):
    return su.Trainer(synth.mlp_init(seed), lr=2e-3, batch=batch, seed=seed, device="cpu")


def test_save_load_round_trip(tmp_path):
    a = _trainer()
    rng = np.random.default_rng(5)
    for t in (a.m, a.v):
        for k in rt.MlpTensors.NAMES:
            getattr(t, k).copy_(torch.as_tensor(rng.standard_normal(rt.MlpTensors.SHAPES[k]).astype(np.float32)))
    a.step = 37
    a.rng.permutation(1000)                     # advance the generator
    path = str(tmp_path / "ckpt.npz")
    a.save(path)
    b = _trainer(seed=9)                        # different weights and generator
    b.load(path)
    assert b.step == 37 and b.lr == a.lr
    for x, y in ((a.w, b.w), (a.m, b.m), (a.v, b.v)):
        hx, hy = x.host(), y.host()
        for k in rt.MlpTensors.NAMES:
            assert np.array_equal(hx[k], hy[k]), k
    # The generators continue identically.
    assert np.array_equal(a.rng.permutation(5000), b.rng.permutation(5000))
    # Plain arrays only: the file loads without pickle.
    with np.load(path, allow_pickle=False) as z:
        assert all(z[n].dtype != object for n in z.files)


def test_load_refuses_other_batch_size(tmp_path):
    a = _trainer(batch=128)
    path = str(tmp_path / "ckpt.npz")
    a.save(path)
    with pytest.raises(ValueError, match="batch"):
        _trainer(batch=256).load(path)
