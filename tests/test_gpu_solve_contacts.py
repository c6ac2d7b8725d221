"""cd_solve_contacts: the force solve alone (Sec. 2.1 sweeps and tests,
Sec. 3.1 domain-wise update) on a caller's contact list, domains and update
order, against the oracle's solve of the same list, partition and order.

The oracle's solve is sequential in the slot order it is given; the library
runs a given order colour by colour (each contact one colour above the
earlier contacts it shares a body with), which must give the same forces bit
for bit."""
import numpy as np
import pytest

from paper_1104_3516_amd import inputs
from tests.test_gpu_parity import _torch

pytestmark = pytest.mark.gpu


def oracle_case(oracle, pk, P, mu=0.3, skin=None):
    if skin is None:
        skin = 2.0 * np.sqrt((pk.v ** 2).sum(0)).max() * 1e-3
    ci, cj = oracle.detect(pk, skin)
    normal, gap, xmid = oracle.geometry(pk, ci, cj)
    tree, dom = oracle.orb(pk.dim, P, pk.box_lo, pk.box_hi, xmid)
    color, slot, ds = oracle.order(pk.n, ci, cj, P, dom)
    return dict(ci=ci, cj=cj, normal=normal, gap=gap, dom=dom, slot=slot, ds=ds, skin=skin)


def oracle_solve(oracle, pk, case, P, slot, ds, R0=None, mu=0.3, **kw):
    params = oracle.make_params(pk.dim, pk.n_walls, mu=mu, n_domains=P, **kw)
    return oracle.solve(params, pk, case["ci"], case["cj"], case["normal"], case["gap"], P, ds,
                        slot, R0=R0)


def gpu_ctx(pk, P, mu=0.3, **kw):
    from paper_1104_3516_amd import binding
    return binding.Context(binding.make_params(pk.dim, pk.n_walls, mu=mu, n_domains=P, **kw), pk,
                           timing=0)


def per_domain_order(dom, ds, key):
    """A domain-major order whose segments sort each domain's contacts by key."""
    order = np.argsort(dom, kind="stable")
    out = []
    for d in range(len(ds) - 1):
        seg = order[ds[d]:ds[d + 1]]
        out.append(seg[np.argsort(key[seg], kind="stable")])
    return np.concatenate(out).astype(np.int32)


@pytest.mark.parametrize("dim,shape,P,kw", [
    (2, (24, 20), 9, dict(max_iter=3000)),
    (2, (40, 33), 17, dict(fixed_iters=37)),
    (3, (10, 9, 7), 6, dict(max_iter=3000)),
])
@pytest.mark.parametrize("which", ["colour_major", "canonical", "random"])
def test_given_list_domains_and_order(oracle, dim, shape, P, kw, which):
    _torch()
    pk = inputs.lattice_2d(*shape, 51) if dim == 2 else inputs.lattice_3d(*shape, 51)
    mu = 0.3 if dim == 2 else 0.5
    case = oracle_case(oracle, pk, P, mu)
    nc = len(case["ci"])
    if which == "colour_major":
        slot = case["slot"]
    elif which == "canonical":
        slot = per_domain_order(case["dom"], case["ds"], np.arange(nc))
    else:
        slot = per_domain_order(case["dom"], case["ds"], np.random.default_rng(5).random(nc))
    R, info, _ = oracle_solve(oracle, pk, case, P, slot, case["ds"], mu=mu, **kw)
    ctx = gpu_ctx(pk, P, mu=mu, **kw)
    res = ctx.solve_contacts(case["ci"], case["cj"], dom=case["dom"], order=slot)
    Rg = ctx.last_R.cpu().numpy()
    assert res.iterations == info.iterations and res.status == info.status
    np.testing.assert_array_equal(Rg, R)
    # the list became the context's current one, with its forces
    c = {k: v.cpu().numpy() for k, v in ctx.contacts().items()}
    np.testing.assert_array_equal(c["R"], R)
    np.testing.assert_array_equal(c["dom"], case["dom"])
    # a given colour-major order is laid out as the library's own
    if which == "colour_major":
        np.testing.assert_array_equal(c["slot"], slot)
    assert res.n_active == int((R[0] > 0).sum())
    assert res.crit_last == pytest.approx(res.n_pass / nc, rel=1e-15)
    dd = (res.r_avg - res.r_avg_prev) ** 2
    ss = (res.r_avg + res.r_avg_prev) ** 2
    assert res.rel_change_last == pytest.approx(dd / ss if ss > 0 else 0.0, rel=1e-12)


@pytest.mark.parametrize("dim", [2, 3])
def test_partition_and_order_from_the_library(oracle, dim):
    """dom = NULL: the contact-count bisection of the mid-gap positions;
    order = NULL: first-fit colour-major order; starting forces given."""
    _torch()
    pk = inputs.lattice_2d(30, 26, 52) if dim == 2 else inputs.lattice_3d(9, 9, 8, 52)
    P = 13
    case = oracle_case(oracle, pk, P)
    nc = len(case["ci"])
    R0 = np.abs(np.random.default_rng(2).normal(size=(dim, nc))) * 0.5
    R, info, _ = oracle_solve(oracle, pk, case, P, case["slot"], case["ds"], R0=R0,
                              max_iter=3000)
    ctx = gpu_ctx(pk, P, max_iter=3000)
    res = ctx.solve_contacts(case["ci"], case["cj"], R=R0)
    assert res.iterations == info.iterations
    np.testing.assert_array_equal(ctx.last_R.cpu().numpy(), R)
    c = {k: v.cpu().numpy() for k, v in ctx.contacts().items()}
    np.testing.assert_array_equal(c["dom"], case["dom"])
    np.testing.assert_array_equal(c["slot"], case["slot"])


def test_mixed_update_and_next_step_warm_start(oracle):
    """The mixed update applies to a given list with the library's own
    order, and a later cd_step warm-starts from the solved list."""
    _torch()
    pk = inputs.lattice_2d(20, 18, 53)
    P = 5
    case = oracle_case(oracle, pk, P)
    par = oracle.parallel_flags(case["ci"], case["cj"], 0.05, 9)
    color, slot, ds = oracle.order(pk.n, case["ci"], case["cj"], P, case["dom"], parallel=par)
    params = oracle.make_params(2, pk.n_walls, n_domains=P, max_iter=3000)
    R, info, _ = oracle.solve(params, pk, case["ci"], case["cj"], case["normal"], case["gap"], P,
                              ds, slot, parallel=par)
    ctx = gpu_ctx(pk, P, max_iter=3000)
    ctx.set_mixed_update(0.05, 9)
    res = ctx.solve_contacts(case["ci"], case["cj"], dom=case["dom"])
    assert res.iterations == info.iterations
    np.testing.assert_array_equal(ctx.last_R.cpu().numpy(), R)
    ctx.set_mixed_update(-1.0)
    ctx.step()          # warm-started from the solved list: runs and converges
    assert ctx.num_contacts() > 0


def test_checks_refuse_bad_inputs(oracle):
    from paper_1104_3516_amd import binding
    _torch()
    pk = inputs.lattice_2d(12, 10, 54)
    case = oracle_case(oracle, pk, 3)
    ci, cj, dom = case["ci"], case["cj"], case["dom"]
    ctx = gpu_ctx(pk, 3)
    bad_lists = [
        (ci[::-1].copy(), cj[::-1].copy()),                 # not canonical
        (cj.copy(), ci.copy()),                              # ci > cj
        (ci, np.where(np.arange(len(cj)) == 3, pk.n + pk.n_walls, cj)),   # no such wall
        (np.where(np.arange(len(ci)) == 0, -1, ci), cj),    # negative id
    ]
    for a, b in bad_lists:
        with pytest.raises(binding.CDError) as e:
            ctx.solve_contacts(a, b)
        assert e.value.code == binding.EINVAL
    with pytest.raises(binding.CDError):
        ctx.solve_contacts(ci, cj, dom=np.where(dom == 0, 3, dom))
    order = case["slot"].copy()
    with pytest.raises(binding.CDError):
        ctx.solve_contacts(ci, cj, order=order)                       # order without dom
    dup = order.copy()
    dup[1] = dup[0]
    with pytest.raises(binding.CDError):
        ctx.solve_contacts(ci, cj, dom=dom, order=dup)
    rev = order[::-1].copy()                                          # domains decreasing
    with pytest.raises(binding.CDError):
        ctx.solve_contacts(ci, cj, dom=dom, order=rev)
    # still usable afterwards
    res = ctx.solve_contacts(ci, cj, dom=dom, order=order)
    assert res.n_contacts == len(ci)
    empty = ctx.solve_contacts(np.zeros(0, np.int32), np.zeros(0, np.int32))
    assert empty.n_contacts == 0 and empty.status == 0


def test_chain_order_needing_many_colours_is_refused(oracle):
    """A chain updated from one end to the other needs one colour per
    contact: more than 64 in one domain is CD_ECAPACITY."""
    from paper_1104_3516_amd import binding
    _torch()
    pk = inputs.chain_2d(80, 1.0)
    ci, cj = oracle.detect(pk, 1e-9, use_cells=False)
    nc = len(ci)
    # contacts along the chain: particle-particle ones in x order, then walls
    pp = np.flatnonzero(cj < pk.n)
    order = np.concatenate([pp, np.flatnonzero(cj >= pk.n)]).astype(np.int32)
    ctx = gpu_ctx(pk, 1)
    with pytest.raises(binding.CDError) as e:
        ctx.solve_contacts(ci, cj, dom=np.zeros(nc, np.int32), order=order)
    assert e.value.code == binding.ECAPACITY


def test_particle_in_more_than_32_domains_is_refused():
    """A particle whose contacts lie in more than 32 domains (the per-particle
    entry limit) is CD_ECAPACITY before any sweep: a star of 40 contacts
    around particle 0, each in a domain of its own.  The context stays
    usable."""
    from paper_1104_3516_amd import binding
    _torch()
    pk = inputs.lattice_2d(8, 6, 95)
    ci = np.zeros(40, np.int32)
    cj = np.arange(1, 41, dtype=np.int32)
    ctx = gpu_ctx(pk, 40)
    with pytest.raises(binding.CDError) as e:
        ctx.solve_contacts(ci, cj, dom=np.arange(40, dtype=np.int32))
    assert e.value.code == binding.ECAPACITY
    assert "32 domains" in str(e.value)
    res = ctx.solve_contacts(ci, cj, dom=np.zeros(40, np.int32))
    assert res.n_contacts == 40 and res.status in (binding.OK, binding.MAXITER)
