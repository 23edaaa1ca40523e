"""GPU parity of the multiresolution transform (Sec. 3.1 details iterated
over levels, Sec. 3.2 lifted coarse values) against the FP64 oracle through
the C ABI: forward element by element, inverse of the oracle's coefficients,
round trips, sizes whose coarse lattice is not a power of two, the full
256^3 x 4 size the benchmark times, graph replay and the argument guards.
Inputs: seeded standard-normal fields (the transform is linear; a smooth
field would leave the fine details near zero and test less)."""
import numpy as np
import pytest

from paper_1912_05371_amd import wacm

from gpu_util import log

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

TOL = {"f64": 1e-12, "f32": 1e-5}
TDT = {"f64": torch.float64, "f32": torch.float32}


def field(n, nf, seed):
    return np.random.default_rng(seed).standard_normal((nf, n, n, n))


def err(a, b):
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("wavelet", [wacm.CDF40, wacm.CDF44])
@pytest.mark.parametrize("n,nlev", [(32, 3), (48, 3), (20, 2), (16, 1)])
def test_mr_matches_oracle(orc, prec, wavelet, n, nlev):
    u = field(n, 4, 100 + n + nlev)
    if prec == "f32":
        u = u.astype(np.float32).astype(np.float64)
    expect = orc.mr_forward(u, nlev, wavelet)
    d = torch.from_numpy(u).to(device="cuda", dtype=TDT[prec])
    work = wacm.mr_work(d)
    wacm.mr_forward(d, nlev, wavelet, work)
    e_fwd = err(d.double().cpu().numpy(), expect)
    # inverse of the oracle's coefficients, against the oracle's inverse
    w = expect.astype(np.float32).astype(np.float64) if prec == "f32" else expect
    back_o = orc.mr_inverse(w, nlev, wavelet)
    d2 = torch.from_numpy(w).to(device="cuda", dtype=TDT[prec])
    wacm.mr_inverse(d2, nlev, wavelet, work)
    e_inv = err(d2.double().cpu().numpy(), back_o)
    # round trip on the device
    wacm.mr_inverse(d, nlev, wavelet, work)
    e_rt = err(d.double().cpu().numpy(), u)
    log(f"mr n={n} nlev={nlev} wavelet={wavelet} {prec}: forward {e_fwd:.2e}, "
        f"inverse {e_inv:.2e}, round trip {e_rt:.2e}")
    assert e_fwd < TOL[prec] and e_inv < TOL[prec] and e_rt < TOL[prec]


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("wavelet", [wacm.CDF40, wacm.CDF44])
def test_mr_full_size(orc, wavelet, prec):
    """256^3 x 4 fields, 5 levels (the benchmark's size): field 1 against the
    oracle element by element (fields are transformed independently, so the
    4-field call must give the 1-field oracle's values there), the 4-field
    round trip to the precision's tolerance."""
    n, nlev = 256, 5
    u = field(n, 4, 7 + wavelet)
    if prec == "f32":
        u = u.astype(np.float32).astype(np.float64)
    log(f"mr full size, wavelet {wavelet}, {prec}: oracle on field 1")
    expect = orc.mr_forward(u[1], nlev, wavelet)
    d = torch.from_numpy(u).to(device="cuda", dtype=TDT[prec])
    work = wacm.mr_work(d)
    wacm.mr_forward(d, nlev, wavelet, work)
    got = d[1].double().cpu().numpy()
    e = err(got, expect)
    wacm.mr_inverse(d, nlev, wavelet, work)
    e_rt = err(d.double().cpu().numpy(), u)
    log(f"  forward field 1 rel err {e:.2e}, round trip {e_rt:.2e}")
    assert e < TOL[prec] and e_rt < TOL[prec]


def test_mr_graph_replay():
    """forward captured in a HIP graph: every replay (with eager copies of
    the input between them) equals the eager call bitwise."""
    n, nlev = 64, 3
    u = torch.from_numpy(field(n, 2, 5)).cuda()
    ref = u.clone()
    work = wacm.mr_work(u)
    wacm.mr_forward(ref, nlev, wacm.CDF44, work)
    buf = u.clone()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    g = torch.cuda.CUDAGraph()
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            wacm.mr_forward(buf, nlev, wacm.CDF44, work)
    torch.cuda.current_stream().wait_stream(s)
    for r in range(3):
        buf.copy_(u)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(buf, ref), f"replay {r}"


def test_mr_guards_and_identity():
    u = torch.from_numpy(field(16, 1, 3)).cuda()
    v = u.clone()
    wacm.mr_forward(v, 0, wacm.CDF44)  # nlev 0: nothing to do, no work needed
    assert torch.equal(u, v)
    with pytest.raises(wacm.WacmError):
        wacm.mr_forward(v, 2, wacm.CDF44)  # CDF 4/4 needs the work buffer
    with pytest.raises(wacm.WacmError):
        wacm.mr_forward(v, 3, wacm.CDF40)  # 16 / 8 < 4
    with pytest.raises(wacm.WacmError):
        wacm.mr_forward(v, 1, 7)  # no such wavelet
    w = torch.from_numpy(field(20, 1, 3)).cuda()
    with pytest.raises(wacm.WacmError):
        wacm.mr_forward(w, 3, wacm.CDF40)  # 20 is not a multiple of 8
    assert torch.equal(u, v)
    # a view starting one element in is not aligned to two elements
    flat = torch.zeros(16 ** 3 + 1, dtype=torch.float64, device="cuda")
    odd = flat[1:].view(1, 16, 16, 16)
    with pytest.raises(wacm.WacmError):
        wacm.mr_forward(odd, 1, wacm.CDF40)
