"""Device-pointer entry points with the host calls' arguments, through the C ABI:
qng_energy_grad_dev (E and grad E in device memory) and qng_step_dev (the
natural-gradient step of Sec. 1, (Re G + eps I) dtheta = -dt grad E, with G,
grad E, E and dtheta in device memory and the shifted solve on the device),
against the FP64 oracle.  Bounds as in the other parity tests: normwise 1e-10
for complex128 G, T, grad E and E; dtheta within max(1e-10, kappa * 1e-14)."""
import sys

import numpy as np
import pytest

import oracle
import workloads as W

pytestmark = pytest.mark.gpu

TOL = 1e-10


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def qng():
    import torch  # noqa: F401
    import paper_2011_02991_amd as q
    return q


@pytest.fixture(scope="module")
def ctx(qng):
    c = qng.Context(0)
    yield c
    c.close()


def rel_err(a, b):
    a, b = np.asarray(a), np.asarray(b)
    return float(np.abs(a - b).max(initial=0.0) / max(np.abs(b).max(initial=0.0), 1e-300))


def cases():
    a = W.config1()
    b = W.scaled(W.config5, 10, 2, n_terms=12)
    b.in_state = W.random_state(10, 71)
    c = W.permute_params(W.scaled(W.config2, 9, 3, n_terms=7), 72)
    return [a, b, c]


@pytest.fixture(scope="module", params=[0, 1, 2], ids=["n10_P80", "n10_P60_in_state", "n9_P54_permuted"])
def case(request):
    return cases()[request.param]


def _dev_in(pr):
    import torch
    if pr.in_state is None:
        return None, None
    t = torch.from_numpy(np.ascontiguousarray(pr.in_state)).to("cuda:0")
    return t, t.data_ptr()


def test_energy_grad_dev(ctx, qng, case):
    import torch
    pr = case
    say(f"case: {pr.name} qng_energy_grad_dev")
    circ = qng.Circuit.from_problem(pr)
    keep, ins = _dev_in(pr)
    E = torch.full((1,), np.nan, dtype=torch.float64, device="cuda:0")
    g = torch.full((pr.n_params,), np.nan, dtype=torch.float64, device="cuda:0")
    ctx.set_stream(torch.cuda.current_stream().cuda_stream)
    try:
        ctx.energy_grad_dev(circ, pr.theta, E.data_ptr(), g.data_ptr(), in_state_dev_ptr=ins)
        torch.cuda.synchronize()
    finally:
        ctx.set_stream(None)
    Eo, go = oracle.energy_grad(pr)
    say(f"{pr.name}: |dE|={abs(E.item() - Eo):.2e} |dgrad|={rel_err(g.cpu().numpy(), go):.2e}")
    assert abs(E.item() - Eo) <= TOL * max(1.0, abs(Eo))
    assert rel_err(g.cpu().numpy(), go) <= TOL
    # the host call gives the same numbers (the same kernels)
    Eh, gh = ctx.energy_grad(circ, pr.theta, in_state=pr.in_state)
    assert Eh == E.item() and np.array_equal(gh, g.cpu().numpy())


@pytest.mark.parametrize("with_G,with_status", [(True, True), (False, False), (False, True)])
def test_step_dev(ctx, qng, case, with_G, with_status):
    import torch
    pr = case
    P = pr.n_params
    say(f"case: {pr.name} qng_step_dev G={with_G} status={with_status}")
    circ = qng.Circuit.from_problem(pr)
    keep, ins = _dev_in(pr)
    dev = torch.device("cuda:0")
    dth = torch.full((P,), np.nan, dtype=torch.float64, device=dev)
    G = torch.full((P, P), np.nan, dtype=torch.complex128, device=dev) if with_G else None
    g = torch.full((P,), np.nan, dtype=torch.float64, device=dev)
    E = torch.full((1,), np.nan, dtype=torch.float64, device=dev)
    st = torch.full((1,), 99, dtype=torch.int32, device=dev) if with_status else None
    ctx.set_stream(torch.cuda.current_stream().cuda_stream)
    try:
        ctx.step_dev(circ, pr.theta, pr.dt, pr.tikhonov, dth.data_ptr(), G.data_ptr() if with_G else None,
                     g.data_ptr(), E.data_ptr(), st.data_ptr() if with_status else None, in_state_dev_ptr=ins)
        torch.cuda.synchronize()
    finally:
        ctx.set_stream(None)
    if with_status:
        assert int(st.item()) == 0
    want = oracle.step(pr)
    kappa = np.linalg.cond(want["G"].real + pr.tikhonov * np.eye(P))
    ed = rel_err(dth.cpu().numpy(), want["dtheta"])
    eg = rel_err(g.cpu().numpy(), want["grad"])
    eE = abs(E.item() - want["E"]) / max(1.0, abs(want["E"]))
    eG = rel_err(G.cpu().numpy(), want["G"]) if with_G else 0.0
    say(f"{pr.name}: |dG|={eG:.2e} |dgrad|={eg:.2e} |dE|={eE:.2e} |ddtheta|={ed:.2e} kappa={kappa:.1e}")
    assert max(eG, eg, eE) <= TOL
    assert ed <= max(TOL, kappa * 1e-14)
    # against the host step (host Cholesky): the same G and gradient, dtheta to rounding
    h = ctx.step(circ, pr.theta, pr.dt, pr.tikhonov, in_state=pr.in_state, want_G=with_G)
    assert np.array_equal(h["grad"], g.cpu().numpy())
    assert rel_err(dth.cpu().numpy(), h["dtheta"]) <= kappa * 1e-14
    if with_G:
        assert np.array_equal(h["G"], G.cpu().numpy())


def test_step_dev_complex64(ctx, qng):
    """complex64 storage (FP64 products and accumulation): the device step
    returns the host step's G and gradient bitwise, dtheta to the solve's rounding."""
    import torch
    pr = W.scaled(W.config3, 12, 2, n_terms=10)
    P = pr.n_params
    circ = qng.Circuit.from_problem(pr)
    dev = torch.device("cuda:0")
    dth = torch.zeros(P, dtype=torch.float64, device=dev)
    G = torch.zeros((P, P), dtype=torch.complex128, device=dev)
    g = torch.zeros(P, dtype=torch.float64, device=dev)
    ctx.set_stream(torch.cuda.current_stream().cuda_stream)
    try:
        ctx.step_dev(circ, pr.theta, pr.dt, pr.tikhonov, dth.data_ptr(), G.data_ptr(), g.data_ptr(), prec="c64")
        torch.cuda.synchronize()
    finally:
        ctx.set_stream(None)
    h = ctx.step(circ, pr.theta, pr.dt, pr.tikhonov, prec="c64")
    kappa = np.linalg.cond(h["G"].real + pr.tikhonov * np.eye(P))
    assert np.array_equal(h["G"], G.cpu().numpy()) and np.array_equal(h["grad"], g.cpu().numpy())
    assert rel_err(dth.cpu().numpy(), h["dtheta"]) <= kappa * 1e-14


@pytest.mark.parametrize("chunk", [0, 8], ids=["all kept", "chunks of 8"])
def test_step_dev_derivative_states(ctx, qng, chunk):
    """The derivative-state variant (QNG_OPT_METHOD = 1, the kept states in
    chunks or all at once) through the device step: the host step's G and
    gradient bitwise, dtheta to the solve's rounding, and the oracle."""
    import torch
    pr = W.scaled(W.config2, 11, 3, n_terms=8)
    P = pr.n_params
    circ = qng.Circuit.from_problem(pr)
    dev = torch.device("cuda:0")
    dth = torch.zeros(P, dtype=torch.float64, device=dev)
    G = torch.zeros((P, P), dtype=torch.complex128, device=dev)
    g = torch.zeros(P, dtype=torch.float64, device=dev)
    ctx.set_option(qng.OPT_METHOD, 1)
    ctx.set_option(qng.OPT_STATE_CHUNK, chunk)
    ctx.set_stream(torch.cuda.current_stream().cuda_stream)
    try:
        ctx.step_dev(circ, pr.theta, pr.dt, pr.tikhonov, dth.data_ptr(), G.data_ptr(), g.data_ptr())
        torch.cuda.synchronize()
        chunks = ctx.stats()["state_chunks"]
        ctx.set_stream(None)
        h = ctx.step(circ, pr.theta, pr.dt, pr.tikhonov)
    finally:
        ctx.set_stream(None)
        ctx.set_option(qng.OPT_METHOD, 0)
        ctx.set_option(qng.OPT_STATE_CHUNK, 0)
    assert chunks == 1 if chunk == 0 else chunks > 1
    want = oracle.step(pr)
    kappa = np.linalg.cond(want["G"].real + pr.tikhonov * np.eye(P))
    assert np.array_equal(h["G"], G.cpu().numpy()) and np.array_equal(h["grad"], g.cpu().numpy())
    assert rel_err(dth.cpu().numpy(), h["dtheta"]) <= kappa * 1e-14
    assert rel_err(G.cpu().numpy(), want["G"]) <= TOL and rel_err(g.cpu().numpy(), want["grad"]) <= TOL
    assert rel_err(dth.cpu().numpy(), want["dtheta"]) <= max(TOL, kappa * 1e-14)


def test_step_dev_not_spd_writes_nothing(ctx, qng):
    """eps = 0 with a zero row of G (a leading RZ on |0>): the device solve
    finds a zero pivot; the status says QNG_E_NOT_SPD and no output changes."""
    import torch
    g = np.array([[W.RZ, 0, -1, 0], [W.RY, 1, -1, 1], [W.CNOT, 1, 0, -1]], dtype=np.int32)
    pr = W.Problem("zrow", 2, g, np.array([0.4, 0.9]), np.array([[3, 3]], np.uint8), np.array([1.0]))
    circ = qng.Circuit.from_problem(pr)
    dev = torch.device("cuda:0")
    outs = [torch.full((2,), 7.0, dtype=torch.float64, device=dev),
            torch.full((2, 2), 7.0, dtype=torch.complex128, device=dev),
            torch.full((2,), 7.0, dtype=torch.float64, device=dev),
            torch.full((1,), 7.0, dtype=torch.float64, device=dev)]
    st = torch.zeros(1, dtype=torch.int32, device=dev)
    ctx.set_stream(torch.cuda.current_stream().cuda_stream)
    try:
        ctx.step_dev(circ, pr.theta, 0.1, 0.0, *[o.data_ptr() for o in outs], st.data_ptr())
        torch.cuda.synchronize()
        assert qng.STATUS[int(st.item())] == "QNG_E_NOT_SPD"
        for o in outs:
            assert torch.all(o == 7.0)
        with pytest.raises(qng.QNGError) as e:
            ctx.step_dev(circ, pr.theta, 0.1, 0.0, *[o.data_ptr() for o in outs])
        assert e.value.name == "QNG_E_NOT_SPD"
        torch.cuda.synchronize()
        for o in outs:
            assert torch.all(o == 7.0)
    finally:
        ctx.set_stream(None)


def test_clone_state_dev(ctx, qng):
    import torch
    for prec, dt in (("c128", torch.complex128), ("c64", torch.complex64)):
        for n in (0, 1, 5, 17):
            src = torch.randn(2 ** n, dtype=dt, device="cuda:0")
            dst = torch.zeros_like(src)
            ctx.clone_state_dev(n, src.data_ptr(), dst.data_ptr(), prec=prec)
            ctx.synchronize()
            assert torch.equal(src, dst)
