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


def test_mr_work_buffer_guards():
    """The binding refuses a CDF 4/4 work buffer that is too small, on another
    device type, or misaligned, before any launch; the field is unchanged."""
    u = torch.from_numpy(field(32, 2, 5)).cuda()
    v = u.clone()
    need = int(wacm.lib().wacm_mr_work_bytes(32, 2, wacm.F64))
    small = torch.empty(need - 256, dtype=torch.uint8, device="cuda")
    with pytest.raises(ValueError):
        wacm.mr_forward(v, 2, wacm.CDF44, small)
    with pytest.raises(ValueError):
        wacm.mr_inverse(v, 2, wacm.CDF44, small)
    with pytest.raises(ValueError):
        wacm.mr_forward(v, 2, wacm.CDF44, torch.empty(need, dtype=torch.uint8))  # host memory
    big = torch.empty(need + 512, dtype=torch.uint8, device="cuda")
    with pytest.raises(ValueError):
        wacm.mr_forward(v, 2, wacm.CDF44, big[8:])  # not 256-byte aligned
    torch.cuda.synchronize()
    assert torch.equal(u, v)
    # the C entry point checks the size itself too
    rc = wacm.lib().wacm_mr_forward(32, 2, wacm.F64, wacm.CDF44, 2, wacm._ptr(v),
                                    wacm._ptr(big), need - 1, None)
    assert rc == wacm.E_INVAL
    torch.cuda.synchronize()
    assert torch.equal(u, v)


def test_mr_maximum_size():
    """n = 1024 (the largest the entry points accept), 8 levels (coarsest
    lattice 4^3), one FP32 field: 4096 sampled finest-level details against
    u - P u written out from the DD4 weights in float64 (the finest level's
    details do not depend on the coarser steps), and the round trip of both
    wavelets to the FP32 tolerance."""
    n, nlev = 1024, 8
    g = torch.Generator(device="cuda")
    g.manual_seed(11)
    u0 = torch.randn((1, n, n, n), dtype=torch.float32, device="cuda", generator=g)
    u = u0.clone()
    work = wacm.mr_work(u)
    log("mr maximum size: n 1024, 8 levels, f32")
    wacm.mr_forward(u, nlev, wacm.CDF40, work)
    rng = np.random.default_rng(5)
    pts = rng.integers(0, n, size=(4096, 3))
    pts = pts[(pts % 2).any(axis=1)]  # odd points of the finest level
    W = np.array([-1.0, 9.0, 9.0, -1.0]) / 16.0
    offs, wts = [], []
    for x, y, z in pts:
        per = []
        for c in (x, y, z):
            per.append([((c + o) % n, w) for o, w in zip((-3, -1, 1, 3), W)] if c % 2 else
                       [(c, 1.0)])
        o_, w_ = [], []
        for zz, wz in per[2]:
            for yy, wy in per[1]:
                for xx, wx in per[0]:
                    o_.append((zz * n + yy) * n + xx)
                    w_.append(wz * wy * wx)
        o_ += [o_[0]] * (64 - len(o_))
        w_ += [0.0] * (64 - len(w_))
        offs.append(o_)
        wts.append(w_)
    flat0 = u0.view(-1)
    nb = torch.as_tensor(np.array(offs), device="cuda")
    vals = flat0[nb].double().cpu().numpy()
    own = np.array([(z * n + y) * n + x for x, y, z in pts])
    ref = flat0[torch.as_tensor(own, device="cuda")].double().cpu().numpy() - \
        np.sum(vals * np.array(wts), axis=1)
    got = u.view(-1)[torch.as_tensor(own, device="cuda")].double().cpu().numpy()
    scale = float(u0.abs().max())
    e_det = float(np.max(np.abs(got - ref))) / scale
    wacm.mr_inverse(u, nlev, wacm.CDF40, work)
    e40 = float((u - u0).abs().max()) / scale
    u.copy_(u0)
    wacm.mr_forward(u, nlev, wacm.CDF44, work)
    wacm.mr_inverse(u, nlev, wacm.CDF44, work)
    e44 = float((u - u0).abs().max()) / scale
    log(f"  {len(pts)} sampled details rel err {e_det:.2e}; round trips {e40:.2e} (CDF 4/0), "
        f"{e44:.2e} (CDF 4/4)")
    assert e_det < 1e-5 and e40 < 1e-5 and e44 < 1e-5
