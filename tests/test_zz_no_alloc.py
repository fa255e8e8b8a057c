"""snap_project_noalloc (static scratch, no caller workspace) against
snap_project (caller workspace), through the C ABI: two calls in a row, the
second on a smaller input, and the size limit."""
import ctypes as C

import numpy as np
import pytest

import synthgen

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_2607_00095_amd as snap  # noqa: E402
from paper_2607_00095_amd.api import STATS_DTYPE, _load  # noqa: E402
from gpu_helpers import to_dev  # noqa: E402


def _lib():
    lib = _load()
    lib.snap_project_noalloc.argtypes = [C.c_void_p] * 7
    lib.snap_project_noalloc.restype = C.c_int
    return lib


def _noalloc(plan, batch):
    uhat, aux = to_dev(batch.uhat), to_dev(batch.aux)
    u = torch.full((plan.total_vars,), np.nan, dtype=torch.float64, device="cuda")
    lam = torch.full((max(plan.total_rows, 1),), np.nan, dtype=torch.float64, device="cuda")
    st = torch.zeros(plan.batch * STATS_DTYPE.itemsize, dtype=torch.uint8, device="cuda")
    s = torch.cuda.current_stream()
    rc = _lib().snap_project_noalloc(plan._h, C.c_void_p(uhat.data_ptr()), C.c_void_p(aux.data_ptr()),
                                     C.c_void_p(u.data_ptr()), C.c_void_p(lam.data_ptr()),
                                     C.c_void_p(st.data_ptr()), C.c_void_p(s.cuda_stream))
    torch.cuda.synchronize()
    return rc, u.cpu().numpy(), lam.cpu().numpy(), snap.stats_to_numpy(st, plan.batch)


def _with_workspace(plan, batch):
    u, lam, st, ws = snap.project(plan, to_dev(batch.uhat), to_dev(batch.aux))
    torch.cuda.synchronize()
    return u.cpu().numpy(), lam.cpu().numpy(), snap.stats_to_numpy(st, plan.batch)


@pytest.mark.parametrize("prec", [snap.PREC_FP64, snap.PREC_MIXED])
def test_noalloc_matches_workspace_entry_point(prec):
    first = synthgen.ragged_batch(batch=6, seed=21, nx_choices=(32, 64), nt_choices=(16, 24))
    second = synthgen.burgers_batch(batch=1, nx=16, nt=6, seed=4)      # smaller input
    for b in (first, second):
        plan = snap.Plan.from_batch(b, snap.Options(precision=prec))
        assert plan.workspace_bytes <= (64 << 20)
        rc, u, lam, st = _noalloc(plan, b)
        assert rc == 0
        u_ref, lam_ref, st_ref = _with_workspace(plan, b)
        assert (st["status"] == 0).all() and (st_ref["status"] == 0).all()
        np.testing.assert_array_equal(u[: b.total_vars], u_ref[: b.total_vars])
        np.testing.assert_array_equal(lam[: b.total_rows], lam_ref[: b.total_rows])
        np.testing.assert_array_equal(st["newton_iters"], st_ref["newton_iters"])


def test_noalloc_rejects_workspace_beyond_the_limit():
    b = synthgen.burgers_batch(batch=4, nx=128, nt=128, seed=1)     # about 84 MB of workspace
    plan = snap.Plan.from_batch(b)
    assert plan.workspace_bytes > (64 << 20)
    rc, u, _, _ = _noalloc(plan, b)
    assert rc == -1
    assert np.isnan(u).all()        # nothing was launched
