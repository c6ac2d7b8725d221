"""Pins of the autograd reference of the fixed-count solve (oracle/torch_ref.py):
its forward equals the C oracle's solve with per-contact friction, and its
gradients equal central differences of itself."""
import numpy as np
import pytest
import torch

from oracle import cdref, torch_ref
from paper_1104_3516_amd import inputs

K = 12


def case(seed=31, nx=10, ny=8, P=3):
    pk = inputs.lattice_2d(nx, ny, seed)
    skin = 0.2 * pk.r.max()
    pb = torch_ref.setup(pk, P, skin)
    mu = inputs.pair_mu(7, pb.ci, pb.cj)
    return pk, pb, mu


def test_forward_equals_c_oracle_with_contact_friction():
    pk, pb, mu = case()
    p = cdref.make_params(2, pk.n_walls, dt=1e-3, fixed_iters=K, n_domains=pb.P, skin=0.2 * pk.r.max())
    R_c, info, _ = cdref.solve(p, pk, pb.ci, pb.cj, pb.normal, pb.gap, pb.P, pb.dom_start, pb.slot,
                               mu_c=mu)
    assert info.iterations == K
    R_t = torch_ref.forces(pb, pk, torch.as_tensor(mu), torch.as_tensor(pk.v),
                           torch.as_tensor(pk.w), K).numpy()
    scale = np.abs(R_c).max()
    assert scale > 0
    assert np.abs(R_t - R_c).max() <= 1e-12 * scale
    # friction mattered: some contacts slide (|R_t| = mu R_n) and some stick
    slide = np.isclose(np.abs(R_c[1]), mu * R_c[0], rtol=1e-12) & (R_c[0] > 0)
    assert slide.any() and (~slide & (R_c[0] > 0)).any()


def test_gradients_equal_central_differences():
    pk, pb, mu = case(seed=33)
    bottom = torch.as_tensor(pb.cj == pk.n + 2)
    mu_t = torch.as_tensor(mu, dtype=torch.float64).requires_grad_(True)
    v_t = torch.as_tensor(pk.v, dtype=torch.float64).requires_grad_(True)
    w_t = torch.as_tensor(pk.w, dtype=torch.float64).requires_grad_(True)

    def loss(m, v, w):
        R = torch_ref.forces(pb, pk, m, v, w, K)
        return R[0][bottom].sum()

    L = loss(mu_t, v_t, w_t)
    gm, gv, gw = torch.autograd.grad(L, [mu_t, v_t, w_t])
    rng = np.random.default_rng(5)
    h = 1e-7
    checked = 0
    for _ in range(4):
        dm = torch.as_tensor(rng.standard_normal(mu.shape))
        dv = torch.as_tensor(rng.standard_normal(pk.v.shape)) * 0.01
        dw = torch.as_tensor(rng.standard_normal(pk.w.shape)) * 0.01
        with torch.no_grad():
            lp = loss(mu_t + h * dm, v_t + h * dv, w_t + h * dw)
            lm = loss(mu_t - h * dm, v_t - h * dv, w_t - h * dw)
        fd = float((lp - lm) / (2 * h))
        an = float((gm * dm).sum() + (gv * dv).sum() + (gw * dw).sum())
        assert abs(fd - an) <= 1e-6 * max(abs(an), 1e-12), (fd, an)
        checked += 1
    assert checked == 4 and float(L) > 0


def _one_disk_on_floor(vx, vy):
    pk = inputs.column_2d(1)
    pk.v = np.array([[vx], [vy]])
    pb = torch_ref.setup(pk, 1, 0.2 * pk.r.max())
    assert len(pb.ci) == 1 and pb.cj[0] == pk.n          # the floor contact
    return pk, pb


def test_disk_hitting_floor_normal_force_derivative():
    """Closed form (Eqs. 3-5): a touching disk moving down at speed U under
    gravity g gets R_n = m (U + g dt)/dt, so dR_n/dv_y = -m/dt."""
    pk, pb = _one_disk_on_floor(0.0, -0.5)
    v = torch.as_tensor(pk.v).requires_grad_(True)
    R = torch_ref.forces(pb, pk, torch.tensor([0.3], dtype=torch.float64), v,
                         torch.as_tensor(pk.w), 1)
    m, dt = pk.m[0], 1e-3
    assert abs(float(R[0, 0]) - m * (0.5 + dt) / dt) <= 1e-12 * m * 0.5 / dt
    (g,) = torch.autograd.grad(R[0, 0], [v])
    assert abs(float(g[1, 0]) + m / dt) <= 1e-12 * m / dt
    assert float(g[0, 0]) == 0.0


def test_sliding_disk_friction_derivative():
    """Sliding (Eqs. 8-9): R_t = -mu R_n sign(u_t), so dR_t/dmu = -R_n sign(u_t);
    sticking: dR_t/dmu = 0."""
    for vx, slides in ((5.0, True), (1e-4, False)):
        pk, pb = _one_disk_on_floor(vx, -0.5)
        mu = torch.tensor([0.3], dtype=torch.float64, requires_grad=True)
        R = torch_ref.forces(pb, pk, mu, torch.as_tensor(pk.v), torch.as_tensor(pk.w), 1)
        (g,) = torch.autograd.grad(R[1, 0], [mu])
        ut_sign = -1.0          # u_t = -(v_x) along t = (1, 0) for the floor contact
        if slides:
            assert abs(float(R[1, 0]) - (-0.3 * float(R[0, 0]) * ut_sign)) <= 1e-12 * float(R[0, 0])
            assert abs(float(g[0]) - (-float(R[0, 0]) * ut_sign)) <= 1e-12 * float(R[0, 0])
        else:
            assert float(g[0]) == 0.0


def test_kept_list_geometry_and_velocities_equal_c_oracle():
    """The multi-step reference's differentiable geometry equals the C
    oracle's normals and gaps, and its velocity update (Eq. 1) equals the C
    oracle's, for arbitrary forces."""
    pk, pb, _ = case(seed=35)
    S = torch_ref._Setup(pb, pk)
    n0, n1, g = torch_ref.geometry(S, torch.as_tensor(pk.x))
    normal, gap, _ = cdref.geometry(pk, pb.ci, pb.cj)
    assert np.abs(n0.numpy() - normal[0]).max() <= 1e-15
    assert np.abs(n1.numpy() - normal[1]).max() <= 1e-15
    assert np.abs(g.numpy() - gap).max() <= 1e-15 * np.abs(pk.x).max()
    rng = np.random.default_rng(8)
    R = rng.standard_normal((2, len(pb.ci)))
    V_c, W_c = cdref.velocities(pk, pb.dt, pb.ci, pb.cj, normal, R)
    V0, V1, W = torch_ref._exchange(S, n0, n1, torch.as_tensor(R[0]), torch.as_tensor(R[1]),
                                    torch.as_tensor(pk.v), torch.as_tensor(pk.w))
    for a, b in ((V0, V_c[0]), (V1, V_c[1]), (W, W_c[0])):
        assert np.abs(a.numpy() - b).max() <= 1e-13 * np.abs(b).max()


def test_kept_list_one_step_equals_single_step():
    pk, pb, mu = case(seed=36)
    args = (torch.as_tensor(mu), torch.as_tensor(pk.v), torch.as_tensor(pk.w))
    R1 = torch_ref.forces(pb, pk, *args, K)
    Rs = torch_ref.forces_steps(pb, pk, *args, 1, K)
    # the geometry differs from the C oracle's only by rounding
    assert float((R1 - Rs).abs().max()) <= 1e-12 * float(R1.abs().max())


def test_falling_disk_two_steps_closed_form():
    """Closed form over two steps (Eqs. 1-5 with the clamped gap): a disk at
    gap g0 above the floor, falling at v_y < 0 under gravity 1, stays open in
    the first step when g0/dt + v_y - dt >= 0 (then v' = v_y - dt and the gap
    becomes g0 + dt v'); in the second it closes when
    s = g0/dt + 2 v_y - 3 dt < 0, with R_n = -m s/dt.  So
    dR_n/dv_y = -2 m/dt: one m/dt through the velocity and one through the
    position update."""
    pk = inputs.column_2d(1)
    g0, vy, dt = 7.5e-4, -0.5, 1e-3
    pk.x[1, 0] += g0
    pk.v = np.array([[0.0], [vy]])
    pb = torch_ref.setup(pk, 1, 0.2 * pk.r.max())
    assert len(pb.ci) == 1 and pb.cj[0] == pk.n
    v = torch.as_tensor(pk.v).requires_grad_(True)
    R = torch_ref.forces_steps(pb, pk, torch.tensor([0.3], dtype=torch.float64), v,
                               torch.as_tensor(pk.w), 2, 3)
    m = pk.m[0]
    s = g0 / dt + 2 * vy - 3 * dt
    assert abs(float(R[0, 0]) - (-m * s / dt)) <= 1e-9 * m * abs(s) / dt
    assert float(R[1, 0]) == 0.0
    (g,) = torch.autograd.grad(R[0, 0], [v])
    assert abs(float(g[1, 0]) + 2 * m / dt) <= 1e-9 * m / dt
    # one step only: still open, no force
    R1 = torch_ref.forces_steps(pb, pk, torch.tensor([0.3], dtype=torch.float64),
                                torch.as_tensor(pk.v), torch.as_tensor(pk.w), 1, 3)
    assert float(R1[0, 0]) == 0.0


def test_kept_list_gradients_equal_central_differences():
    pk, pb, mu = case(seed=37)
    bottom = torch.as_tensor(pb.cj == pk.n + 2)
    mu_t = torch.as_tensor(mu, dtype=torch.float64).requires_grad_(True)
    v_t = torch.as_tensor(pk.v, dtype=torch.float64).requires_grad_(True)
    w_t = torch.as_tensor(pk.w, dtype=torch.float64).requires_grad_(True)

    def loss(m, v, w):
        return torch_ref.forces_steps(pb, pk, m, v, w, 3, 8)[0][bottom].sum()

    L = loss(mu_t, v_t, w_t)
    gm, gv, gw = torch.autograd.grad(L, [mu_t, v_t, w_t])
    rng = np.random.default_rng(6)
    h = 1e-7
    for _ in range(3):
        dm = torch.as_tensor(rng.standard_normal(mu.shape))
        dv = torch.as_tensor(rng.standard_normal(pk.v.shape)) * 0.01
        dw = torch.as_tensor(rng.standard_normal(pk.w.shape)) * 0.01
        with torch.no_grad():
            lp = loss(mu_t + h * dm, v_t + h * dv, w_t + h * dw)
            lm = loss(mu_t - h * dm, v_t - h * dv, w_t - h * dw)
        fd = float((lp - lm) / (2 * h))
        an = float((gm * dm).sum() + (gv * dv).sum() + (gw * dw).sum())
        assert abs(fd - an) <= 1e-6 * max(abs(an), 1e-12), (fd, an)
    assert float(L) > 0
