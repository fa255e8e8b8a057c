"""GPU parity of the Burgers boundary-row family (Dirichlet on the left,
Riemann-sum mass, Neumann on the right, one closed-form Schur solve per time
slab) against the oracle: forward, multipliers and adjoint, element-wise."""
import numpy as np
import pytest

import synthgen
from oracle.families import family_of
from oracle.kkt import adjoint_sample

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_2607_00095_amd as snap  # noqa: E402
from gpu_helpers import check_samples, gpu_backward, gpu_project, oracle_solution, rel_err  # noqa: E402

# every launch class on both sides of its edges (16-lane groups with 1, 2, 4
# or 8 x registers per lane up to nx = 128, whole-wavefront groups with 4 or 8
# above), the smallest grid, one time step, and slab counts that do not fill
# the eight wavefronts evenly
CASES = [(3, 1), (4, 2), (16, 3), (17, 4), (32, 6), (33, 2), (64, 3), (65, 7), (101, 101), (128, 3), (129, 2),
         (200, 13), (256, 3), (257, 2), (333, 9), (512, 5)]


@pytest.mark.parametrize("nx,nt", CASES)
def test_boundary_rows_match_oracle(nx, nt):
    b = synthgen.burgers_bc_batch(batch=3, nx=nx, nt=nt, seed=11 * nx + nt)
    res = gpu_project(b)
    check_samples(b, res, [0, 1, 2], 1e-10, 1e-8)


def test_boundary_rows_ragged_batch():
    rng = np.random.default_rng(5)
    samples = []
    for i in range(12):
        nx, nt = int(rng.integers(3, 300)), int(rng.integers(1, 40))
        samples += synthgen.burgers_bc_batch(batch=1, nx=nx, nt=nt, seed=100 + i).samples
    b = synthgen.Batch(samples, name="bc_ragged").pack()
    res = gpu_project(b)
    check_samples(b, res, range(len(b)), 1e-10, 1e-8)


def test_boundary_rows_full_config_sampled():
    b = synthgen.make("burgers_bc")
    res = gpu_project(b)
    st = res["stats"]
    assert (st["status"] == 0).all(), np.unique(st["status"], return_counts=True)
    assert st["h_inf"].max() <= 1e-8
    check_samples(b, res, [0, 1, 255, 511], 1e-10, 1e-8)


@pytest.mark.parametrize("nx,nt", [(3, 2), (4, 3), (101, 11), (300, 6)])
def test_boundary_rows_adjoint_matches_oracle(nx, nt):
    # (at nx = 3 the rows fix every variable: the gradient is zero up to rounding)
    b = synthgen.burgers_bc_batch(batch=2, nx=nx, nt=nt, seed=nx + nt)
    res = gpu_project(b)
    grad = synthgen.upstream_grad(b, seed=3)
    g, st = gpu_backward(res, grad)
    assert (st["status"] == 0).all()
    for s, smp in enumerate(b.samples):
        vo = b.var_off[s]
        u_o, lam_o = oracle_solution(smp)
        g_o = adjoint_sample(family_of(smp), u_o, lam_o, grad[vo:vo + smp.n])
        scale = np.abs(grad[vo:vo + smp.n]).max()
        assert np.abs(g[vo:vo + smp.n] - g_o).max() <= 1e-12 * scale
        if nx > 3:
            assert rel_err(g[vo:vo + smp.n], g_o) <= 1e-12


def test_boundary_rows_feasible_input_is_a_fixed_point():
    # project twice: the second call starts on the constraint set
    b = synthgen.burgers_bc_batch(batch=2, nx=50, nt=4, seed=2)
    res = gpu_project(b)
    b2 = synthgen.Batch([synthgen.Sample(s.family, s.nx, 1, s.nt, s.dt, s.dx,
                                         uhat=res["u_np"][o:o + s.n].reshape(s.nt, s.nx), aux=s.aux)
                         for s, o in zip(b.samples, b.var_off)]).pack()
    res2 = gpu_project(b2)
    np.testing.assert_allclose(res2["u_np"], res["u_np"], rtol=0, atol=1e-13)
    assert np.abs(res2["lam_np"]).max() <= 1e-10


def test_boundary_rows_mixed_option_and_nonfinite():
    b = synthgen.burgers_bc_batch(batch=2, nx=40, nt=3, seed=4)
    r64 = gpu_project(b)
    r32 = gpu_project(b, snap.Options(precision=snap.PREC_MIXED))
    np.testing.assert_array_equal(r64["u_np"], r32["u_np"])
    b.uhat[5] = np.nan
    bad = gpu_project(b)
    assert bad["stats"]["status"][0] == 3 and bad["stats"]["status"][1] == 0


@pytest.mark.parametrize("nx", [2, 513])
def test_boundary_rows_unsupported_grids(nx):
    b = synthgen.burgers_bc_batch(batch=1, nx=max(nx, 3), nt=2, seed=1)
    b.samples[0].nx = nx
    with pytest.raises(snap.SnapError):
        snap.Plan.from_batch(b)
