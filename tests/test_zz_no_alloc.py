"""The allocation-free scheduler inference entry point (mf_model_forward_noalloc)
against the allocating one (mf_model_forward), through the C ABI: the same
kernels on the same inputs give the same logits bit for bit, on two calls in a
row (the second on a smaller grid, so the shared device array holds the first
call's activations), in BF16 and FP32; a grid beyond the array's limit is
rejected."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mf():
    from paper_1109_1146_amd import mf as _mf
    _mf.load()
    return _mf


def test_noalloc_forward_matches_forward(mf):
    torch = pytest.importorskip("torch")
    m = mf.Model(16, seed=7)
    rng = np.random.default_rng(11)
    for bf16 in (True, False):
        for dims in ((8, 9, 10), (3, 5, 4)):
            nv = int(np.prod(dims))
            x = torch.from_numpy(rng.random((nv, 6), dtype=np.float32)).cuda()
            want = m.forward(x, dims, bf16=bf16)
            out = torch.full((nv,), float("nan"), dtype=torch.float32, device="cuda")
            m.forward_noalloc(x, out, dims, bf16=bf16)
            torch.cuda.synchronize()
            print(f"noalloc forward dims={dims} bf16={bf16}", flush=True)
            assert torch.equal(out, want)
    # 2 * 16 channels * voxels must fit the 2^20 floats of the array
    big = (32, 32, 33)
    x = torch.zeros((int(np.prod(big)), 6), dtype=torch.float32, device="cuda")
    out = torch.zeros(int(np.prod(big)), dtype=torch.float32, device="cuda")
    with pytest.raises(mf.MFError) as e:
        m.forward_noalloc(x, out, big)
    assert e.value.status == mf.MF_E_INVAL
    m.close()
