"""GPU: the S' evaluation (GQ_SP, the normal derivative of the single layer potential) against
the oracle, and the exterior Neumann integral equation of Sec. 1 (eq. ext-neumann-ie) solved by
batched GMRES over the library's evaluation.

Error measure as in test_gpu_parity: max |gpu - oracle| / max |oracle|. S' uses the expansions
of S (the same FMM error budget: 1e-10 at p_fmm 30) differentiated at the targets."""
import copy

import numpy as np
import pytest

import gq_inputs as gi
import oracle

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _rel(a, b):
    return float(np.abs(a - b).max() / np.abs(b).max())


def _dev(x):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float64, device="cuda:0")


def _ctx(geom, nrm=None, **params):
    from paper_1801_04070_amd import QBXFMM
    q = QBXFMM(device=0)
    q.set_geometry_from(geom)
    q.build(**params)
    if nrm is not None:
        q.set_target_normals(nrm)
    return q


@pytest.fixture(scope="module")
def c1():
    return gi.starfish_c1()


def test_sp_requires_target_normals(c1):
    from paper_1801_04070_amd import GQ_SP, GQError
    q = _ctx(c1, p_qbx=8, p_fmm=15)
    with pytest.raises(GQError):
        q.eval(GQ_SP, _dev(gi.fourier_density(c1, seed=0)))
    with pytest.raises(GQError):
        q.set_target_normals(c1.src_nrm[:-1])


@pytest.mark.parametrize("direct", [False, True])
def test_sp_matches_oracle_c1(c1, direct):
    from paper_1801_04070_amd import GQ_SP
    mu = gi.fourier_density(c1, seed=0)
    q = _ctx(c1, c1.src_nrm, p_qbx=8, p_fmm=30)
    gpu = q.eval(GQ_SP, _dev(mu), direct=direct).cpu().numpy()
    ref = oracle.qbx_normal_derivative(c1, mu, p_qbx=8, tgt_nrm=c1.src_nrm)
    err = _rel(gpu, ref)
    print(f"S' C1 direct={direct} rel_err={err:.3e}")
    assert err < (1e-12 if direct else 1e-10)


def test_sp_batch_on_matrix_cores_and_point_targets():
    """8 densities (the batched kernels) against one-density evaluations and the oracle, on
    three stars with a few off-surface point targets (no center: the differentiated expansion
    of the internal point center)."""
    from paper_1801_04070_amd import GQ_SP
    g = gi.random_stars(n_curves=3, panels_per_curve=128, seed=3)
    g = copy.copy(g)
    extra = np.array([[g.src_xy[:, 0].mean() + 0.37, g.src_xy[:, 1].max() + 1.1],
                      [g.src_xy[:, 0].min() - 0.9, g.src_xy[:, 1].mean() - 0.2]])
    g.tgt_xy = np.concatenate([g.tgt_xy, extra])
    g.tgt_ctr = np.concatenate([g.tgt_ctr, np.full((2, 2), -1, dtype=np.int32)])
    nrm = np.concatenate([g.src_nrm, np.array([[0.6, 0.8], [-1.0, 0.0]])])
    dens = np.stack([gi.fourier_density(g, seed=40 + j) for j in range(8)])
    q = _ctx(g, nrm, p_qbx=10, p_fmm=30)
    batch = q.eval(GQ_SP, _dev(dens)).cpu().numpy()
    one = q.eval(GQ_SP, _dev(dens[5])).cpu().numpy()
    assert _rel(batch[5], one) < 1e-13
    ref = oracle.qbx_normal_derivative(g, dens[5], p_qbx=10, tgt_nrm=nrm)
    err = _rel(batch[5], ref)
    print(f"S' batch of 8 rel_err={err:.3e}, point targets {np.abs(batch[5][-2:] - ref[-2:]).max():.2e}")
    assert err < 1e-10
    assert np.abs(batch[5][-2:] - ref[-2:]).max() < 1e-10 * np.abs(ref).max()


def test_sp_full_size_sampled():
    """The 131072-source workload, S' at 512 sampled targets against the oracle (1e-10)."""
    from paper_1801_04070_amd import GQ_SP
    g = gi.config_geometry("c2")
    mu = gi.fourier_density(g, seed=4)
    q = _ctx(g, g.src_nrm, p_qbx=12, p_fmm=30)
    gpu = q.eval(GQ_SP, _dev(mu)).cpu().numpy()
    idx = np.random.default_rng(11).choice(g.n_tgt, 512, replace=False)
    ref = oracle.qbx_normal_derivative(g, mu, p_qbx=12, tgt_xy=g.tgt_xy[idx],
                                       tgt_nrm=g.src_nrm[idx], tgt_ctr=g.tgt_ctr[idx])
    err = _rel(gpu[idx], ref)
    print(f"S' full size rel_err={err:.3e}")
    assert err < 1e-10


def test_exterior_neumann_gmres_matches_oracle_solve():
    """-mu/2 + S' mu = g on the starfish (2048 nodes) with the Neumann data of point charges
    inside: GMRES over the GPU evaluation converges like the oracle-driven solve, its density
    matches that solve's, and S mu at check points outside (point targets of a second context)
    reproduces the manufactured field to the discretization's accuracy."""
    from paper_1801_04070_amd import GQ_S, QBXFMM
    from paper_1801_04070_amd.bie import gmres, neumann_operator
    g = gi.discretize([gi.StarCurve(amp=0.25, arms=5)], 128, order=16)
    rhs, xc, uc = gi.neumann_test_problem(g, seed=5)
    q = _ctx(g, g.src_nrm, p_qbx=10, p_fmm=30)
    x, its, res = gmres(neumann_operator(q), _dev(rhs)[None, :], tol=1e-12, maxiter=40)
    torch.cuda.synchronize()
    mu = x[0].cpu().numpy()

    def apply_oracle(m):
        out = np.stack([oracle.qbx_normal_derivative(g, r.numpy(), p_qbx=10, tgt_nrm=g.src_nrm)
                        for r in m])
        return -0.5 * m + torch.as_tensor(out)

    xo, its_o, _ = gmres(apply_oracle, torch.as_tensor(rhs)[None, :], tol=1e-12, maxiter=40)
    dmu = _rel(mu, xo[0].numpy())
    ev = copy.copy(g)
    ev.tgt_xy, ev.tgt_ctr = xc, np.full((len(xc), 2), -1, dtype=np.int32)
    qe = QBXFMM(device=0)
    qe.set_geometry_from(ev)
    qe.build(p_qbx=10, p_fmm=30)
    u = qe.eval(GQ_S, _dev(mu)).cpu().numpy()
    err = np.abs(u - uc).max() / np.abs(uc).max()
    print(f"GMRES {its[0]} iterations (oracle {its_o[0]}), residual {res[0]:.1e}, "
          f"density vs oracle solve {dmu:.1e}, BVP error {err:.2e}")
    assert its[0] <= 20 and abs(int(its[0]) - int(its_o[0])) <= 1 and res[0] <= 1e-12
    assert dmu < 1e-9
    assert err < 1e-6


def test_exterior_neumann_many_right_hand_sides():
    """8 right-hand sides (charge sets of 8 seeds) in one batched GMRES: each solution equals the
    solution of its own one-right-hand-side solve."""
    from paper_1801_04070_amd.bie import gmres, neumann_operator
    g = gi.discretize([gi.StarCurve(amp=0.25, arms=5)], 128, order=16)
    rhs = np.stack([gi.neumann_test_problem(g, seed=20 + j)[0] for j in range(8)])
    q = _ctx(g, g.src_nrm, p_qbx=10, p_fmm=30)
    op = neumann_operator(q)
    xb, its_b, res_b = gmres(op, _dev(rhs), tol=1e-12, maxiter=40)
    x3, its_3, _ = gmres(op, _dev(rhs[3])[None, :], tol=1e-12, maxiter=40)
    torch.cuda.synchronize()
    assert (res_b <= 1e-12).all() and its_b.max() <= 20
    assert _rel(xb[3].cpu().numpy(), x3[0].cpu().numpy()) < 1e-10
