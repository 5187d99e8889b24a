"""pip_plan_create (one creator for every plan kind, descriptors holding the
typed creators' arguments) against the eager calls: the plans it returns
autotune, launch and give the same labels, counts and costs bit for bit;
unknown kinds and NULL descriptors are refused."""
from __future__ import annotations

import ctypes
import sys

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def P():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2007_15385_amd as P
    P.load_library()
    return P


def run_plan(P, h):
    from paper_2007_15385_amd.api import _lib
    s = torch.cuda.current_stream().cuda_stream
    assert _lib().pip_plan_autotune(h, 2, s) == 0
    assert _lib().pip_plan_launch(h, s) == 0
    torch.cuda.synchronize()
    _lib().pip_plan_destroy(h)


def test_plan_create_batched(P):
    B = W.uneven_batch(P=64, size_lo=100, size_hi=5000)
    t = [torch.from_numpy(a).cuda() for a in (B.vtx_off, B.V, B.pt_off, B.Q, B.lbl_word_off)]
    want, _, _ = P.pip_voronoi_batched(*t)
    labels = torch.full_like(want, -1)
    status = torch.full((B.num_polygons,), -7, dtype=torch.int32, device="cuda")
    d = P.BatchedDesc(B.num_polygons, t[0].data_ptr(), t[1].data_ptr(), t[1].shape[0],
                      t[2].data_ptr(), t[3].data_ptr(), t[3].shape[0], t[4].data_ptr(),
                      labels.data_ptr(), status.data_ptr())
    say("[case] pip_plan_create batched")
    run_plan(P, P.pip_plan_create(P.PIP_PLAN_BATCHED, d))
    assert torch.equal(labels, want)
    assert (status.cpu().numpy() == 0).all()


def test_plan_create_allpairs(P):
    F = torch.from_numpy(W.car_footprint()).cuda()
    poses, cs = W.random_poses(100, extent=10.0)
    Vw = P.pip_poses_to_polygons(F, torch.from_numpy(poses).cuda(), torch.from_numpy(cs).cuda())
    rng = np.random.default_rng(5)
    Q = torch.from_numpy(rng.uniform(-12, 12, size=(4001, 2)).astype(np.float32)).cuda()
    want_l, want_c, _ = P.pip_voronoi_allpairs(Vw, Q)
    labels = torch.full_like(want_l, -1)
    counts = torch.full_like(want_c, -1)
    d = P.AllpairsDesc(Vw.shape[0], Vw.shape[1], Vw.data_ptr(), Q.data_ptr(), Q.shape[0],
                       labels.data_ptr(), counts.data_ptr(), None)
    say("[case] pip_plan_create all pairs")
    run_plan(P, P.pip_plan_create(P.PIP_PLAN_ALLPAIRS, d))
    assert torch.equal(labels, want_l) and torch.equal(counts, want_c)


def test_plan_create_cost(P):
    F = torch.from_numpy(W.car_footprint().astype(np.float32)).cuda()
    rng = np.random.default_rng(6)
    K = 300
    poses = np.stack([rng.uniform(-5, 5, K), rng.uniform(-5, 5, K), rng.uniform(-3, 3, K)],
                     1).astype(np.float32)
    Pt = torch.from_numpy(poses).cuda()
    Q = torch.from_numpy(rng.uniform(-8, 8, size=(3000, 2)).astype(np.float32)).cuda()
    want = P.pip_cost_fwd(F, Pt, Q)
    cost = torch.full((K,), -1.0, dtype=torch.float32, device="cuda")
    d = P.CostDesc(F.data_ptr(), F.shape[0], Pt.data_ptr(), K, Q.data_ptr(), Q.shape[0],
                   cost.data_ptr(), None, None, None, None)
    say("[case] pip_plan_create cost forward")
    run_plan(P, P.pip_plan_create(P.PIP_PLAN_COST_FWD, d))
    assert torch.equal(cost, want)
    g = torch.from_numpy(rng.uniform(0.5, 2.0, K).astype(np.float32)).cuda()
    want_gp, want_gf, _ = P.pip_cost_bwd(F, Pt, Q, g)
    gp = torch.empty((K, 3), dtype=torch.float32, device="cuda")
    gf = torch.empty_like(F)
    d = P.CostDesc(F.data_ptr(), F.shape[0], Pt.data_ptr(), K, Q.data_ptr(), Q.shape[0], None,
                   g.data_ptr(), gp.data_ptr(), gf.data_ptr(), None)
    say("[case] pip_plan_create cost backward")
    run_plan(P, P.pip_plan_create(P.PIP_PLAN_COST_BWD, d))
    assert torch.equal(gp, want_gp) and torch.equal(gf, want_gf)


def test_plan_create_refuses_bad_kind_and_desc(P):
    d = P.AllpairsDesc()
    with pytest.raises(P.PipError):
        P.pip_plan_create(7, d)
    from paper_2007_15385_amd.api import _lib, context
    h = ctypes.c_void_p()
    assert _lib().pip_plan_create(context(0), 0, None, ctypes.byref(h)) == 1
