"""The adjoint entry point that allocates nothing (qs_adjoint_backward_noalloc)
against the allocating qs_adjoint_backward, through the C ABI, on two calls
in a row (the second with a smaller batch), plus its refusals: a shape with
no cached plan, a path other than the register/LDS engine, partial sums
larger than its device array."""
import numpy as np
import pytest

from workloads import circuits as C
from workloads import data as Dt

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if torch.cuda.is_available():
    from paper_2509_25075_amd import _native as N
    from paper_2509_25075_amd import sim

TOL = {"c64": 1e-4, "c128": 1e-10}


def _announce(msg):
    print(msg, flush=True)


def _dev(a, dt):
    return None if a is None else torch.as_tensor(np.asarray(a)).to("cuda", dt).contiguous()


def _both(s, w, B, rng, per_sample=False):
    """Forward once, then the adjoint through both entry points on the same
    final state; returns the two (grad_params, grad_feats) pairs."""
    n = s.n
    rd = s.rdtype
    P = s.h.n_params
    params = rng.uniform(-np.pi, np.pi, (B, P) if per_sample else P)
    pt = _dev(params, rd)
    ft = _dev(rng.uniform(-1, 1, (B, s.h.n_features)), rd) if s.h.n_features else None
    if w.encoding == "amplitude":
        st = s.encode_amplitude(_dev(rng.standard_normal((B, 1 << n)), rd))
    else:
        st = s.zero_state(B)
    s.forward(pt, ft, st, want_expz=False)
    dz = _dev(rng.uniform(-1, 1, (B, n)), torch.float64)
    gshape = (B, P) if per_sample else (P,)
    out = []
    for fn in ("alloc", "noalloc"):
        gp = torch.full(gshape, 7.0, dtype=torch.float64, device="cuda")
        gf = (torch.full((B, s.h.n_features), 7.0, dtype=torch.float64, device="cuda")
              if s.h.n_features else None)
        if fn == "alloc":
            N.qs_adjoint_backward(s.h, s.qs_dtype, pt, ft, st, dexpz=dz, grad_params=gp,
                                  grad_feats=gf, ws=s.workspace(B), flags=s.flags)
        else:
            N.qs_adjoint_backward_noalloc(s.h, s.qs_dtype, pt, ft, st, dexpz=dz,
                                          grad_params=gp, grad_feats=gf, flags=s.flags)
        out.append((gp, gf))
    torch.cuda.synchronize()
    return out


@pytest.mark.parametrize("key,dtype,B1,B2", [("c2", "c64", 512, 96), ("c3", "c64", 700, 65),
                                             ("c2", "c128", 64, 10), ("c4", "c64", 128, 33)])
def test_noalloc_adjoint_matches_the_allocating_call_twice(key, dtype, B1, B2):
    w = Dt.make_workload(key, 4)
    s = sim.Simulator(w.circuit, dtype)
    rng = np.random.default_rng(77)
    for B in (B1, B2):  # the second call has a smaller batch
        _announce(f"noalloc {key} {dtype} B={B}")
        assert N.qs_workspace_size(s.h, s.qs_dtype, B) <= N.QS_NOALLOC_SCRATCH_BYTES
        (ga, fa), (gn, fn) = _both(s, w, B, rng)
        np.testing.assert_allclose(gn.cpu().numpy(), ga.cpu().numpy(), atol=TOL[dtype], rtol=0)
        if fa is not None:
            np.testing.assert_allclose(fn.cpu().numpy(), fa.cpu().numpy(), atol=TOL[dtype],
                                       rtol=0)


def test_noalloc_adjoint_per_sample_params():
    c = C.hea_ry_rz_ring(9, 3)
    w = Dt.Workload("hea n9", 9, 1, c, "c64", "amplitude", "weighted_z")
    s = sim.Simulator(c, "c64", N.QS_FLAG_PER_SAMPLE_PARAMS)
    rng = np.random.default_rng(78)
    for B in (40, 7):
        _announce(f"noalloc per-sample B={B}")
        (ga, _), (gn, _) = _both(s, w, B, rng, per_sample=True)
        np.testing.assert_allclose(gn.cpu().numpy(), ga.cpu().numpy(), atol=1e-4, rtol=0)


def test_noalloc_adjoint_refusals():
    rng = np.random.default_rng(79)
    # a circuit no call has planned yet
    c = C.hea_ry_rz_ring(8, 2)
    c.gates["scale"] = np.where(np.isin(c.gates["op"], list(C.ROTATIONS)), 0.613, 1.0)
    h = N.CircuitHandle(c)
    st = torch.zeros(4, 256, dtype=torch.complex64, device="cuda")
    st[:, 0] = 1
    p = torch.zeros(c.n_params, device="cuda")
    gp = torch.empty(c.n_params, dtype=torch.float64, device="cuda")
    dz = torch.zeros(4, 8, dtype=torch.float64, device="cuda")
    with pytest.raises(N.QsError) as e:
        N.qs_adjoint_backward_noalloc(h, N.QS_C64, p, None, st, dexpz=dz, grad_params=gp)
    assert e.value.status == N.QS_ERR_NOT_PLANNED
    # the large-state path needs state-sized workspace: not this entry point
    c15 = C.hea_ry_rz_ring(15, 1)
    st15 = torch.zeros(1, 1 << 15, dtype=torch.complex64, device="cuda")
    with pytest.raises(N.QsError) as e:
        N.qs_adjoint_backward_noalloc(
            N.CircuitHandle(c15), N.QS_C64, torch.zeros(c15.n_params, device="cuda"), None,
            st15, dexpz=torch.zeros(1, 15, dtype=torch.float64, device="cuda"),
            grad_params=torch.empty(c15.n_params, dtype=torch.float64, device="cuda"))
    assert e.value.status == N.QS_ERR_UNSUPPORTED
    # partial sums beyond the device array: rejected before any work
    w = Dt.make_workload("c3", 4)
    B = 131072
    hb = N.CircuitHandle(w.circuit)
    assert N.qs_workspace_size(hb, N.QS_C128, B) > N.QS_NOALLOC_SCRATCH_BYTES
    big = torch.zeros(B, 256, dtype=torch.complex128, device="cuda")
    with pytest.raises(N.QsError) as e:
        N.qs_adjoint_backward_noalloc(
            hb, N.QS_C128, torch.zeros(w.circuit.n_params, dtype=torch.float64, device="cuda"),
            torch.zeros(B, 4, dtype=torch.float64, device="cuda"), big,
            dexpz=torch.zeros(B, 8, dtype=torch.float64, device="cuda"),
            grad_params=torch.empty(w.circuit.n_params, dtype=torch.float64, device="cuda"))
    assert e.value.status == N.QS_ERR_WORKSPACE
    del big
    torch.cuda.synchronize()
    # after planning it through the allocating call, the same shape runs
    s = sim.Simulator(c, "c64")
    gp2, _ = s.adjoint(p, None, st, dexpz=dz)
    N.qs_adjoint_backward_noalloc(h, N.QS_C64, p, None, st, dexpz=dz, grad_params=gp)
    torch.cuda.synchronize()
    np.testing.assert_allclose(gp.cpu().numpy(), gp2.cpu().numpy(), atol=1e-4, rtol=0)
    assert rng is not None
