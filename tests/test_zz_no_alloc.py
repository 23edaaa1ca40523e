"""wacm_mr_forward_noalloc (the multiresolution transform whose CDF 4/4 work
buffer is the library's static device scratch array) against wacm_mr_forward
with a caller work buffer, through the C ABI: the same kernels, so the
results must agree bit for bit.  Two calls in a row on different sizes (the
second smaller, so it runs on scratch contents left by the first), both
precisions and both wavelets, the largest FP64 size the scratch admits, and
a size above it rejected before any launch."""
import numpy as np
import pytest

from paper_1912_05371_amd import wacm

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def field(n, nf, seed, dtype):
    rng = np.random.default_rng(seed)
    return torch.from_numpy(rng.standard_normal((nf, n, n, n))).to("cuda", dtype)


def reference(u, nlev, wavelet):
    r = u.clone()
    wacm.mr_forward(r, nlev, wavelet, wacm.mr_work(r))
    return r


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("wavelet", [wacm.CDF44, wacm.CDF40])
def test_noalloc_matches_forward_twice(dtype, wavelet):
    print(f"noalloc {dtype} wavelet {wavelet}", flush=True)
    for k, (n, nf, nlev) in enumerate(((64, 4, 3), (32, 2, 2))):
        u = field(n, nf, 10 + k, dtype)
        ref = reference(u, nlev, wavelet)
        v = u.clone()
        wacm.mr_forward_noalloc(v, nlev, wavelet)
        torch.cuda.synchronize()
        assert torch.equal(v, ref), (n, nf, nlev)
        assert not torch.equal(v, u)


def test_noalloc_largest_fp64_size_and_limit():
    print("noalloc limit", flush=True)
    n, nf = 128, 4
    need = int(wacm.lib().wacm_mr_work_bytes(n, nf, wacm.F64))
    assert need <= wacm.MR_SCRATCH_BYTES
    u = field(n, nf, 3, torch.float64)
    ref = reference(u, 4, wacm.CDF44)
    v = u.clone()
    wacm.mr_forward_noalloc(v, 4, wacm.CDF44)
    torch.cuda.synchronize()
    assert torch.equal(v, ref)
    # above the scratch size: rejected, nothing written
    big = field(256, 2, 4, torch.float64)
    assert int(wacm.lib().wacm_mr_work_bytes(256, 2, wacm.F64)) > wacm.MR_SCRATCH_BYTES
    keep = big.clone()
    with pytest.raises(wacm.WacmError) as ei:
        wacm.mr_forward_noalloc(big, 3, wacm.CDF44)
    assert ei.value.code == wacm.E_INVAL
    torch.cuda.synchronize()
    assert torch.equal(big, keep)
    # CDF 4/0 needs no work buffer: any valid size runs
    ref40 = reference(big, 3, wacm.CDF40)
    wacm.mr_forward_noalloc(big, 3, wacm.CDF40)
    torch.cuda.synchronize()
    assert torch.equal(big, ref40)
