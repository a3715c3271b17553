"""pds_kmeans_step_noalloc (the K-means iteration for callers that cannot
allocate) against pds_kmeans_step with a caller workspace, through the C ABI:
two calls in a row on the library's scratch array, the second with a smaller
input, each compared with the workspace call on the same inputs (assignments,
centers and objective bit for bit: every sum is fixed point), for FP32 and
FP64 plans; and the
size limit is reported as a workspace error before any launch."""
import ctypes

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import paper_1511_00152_amd as pds  # noqa: E402
from paper_1511_00152_amd import _lib  # noqa: E402
import synth  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def device():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)


def _p(t):
    return ctypes.c_void_p(t.data_ptr())


def _both(plan, vals, idx, centers):
    """One round through each entry point on the same inputs."""
    L = pds.lib()
    n, K = vals.shape[0], centers.shape[0]
    dev = vals.device
    s = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    out_w = torch.full_like(centers, float("nan"))
    out_s = torch.full_like(centers, float("nan"))
    a_w = torch.full((n,), -7, dtype=torch.int32, device=dev)
    a_s = torch.full((n,), -7, dtype=torch.int32, device=dev)
    j_w = torch.zeros(1, dtype=torch.float64, device=dev)
    j_s = torch.zeros(1, dtype=torch.float64, device=dev)
    ws = plan.workspace(pds.PDS_OP_KMEANS, n, K, device=dev)
    _lib.check(L.pds_kmeans_step(plan.handle, _p(vals), _p(idx), n, K, _p(centers), _p(out_w), _p(a_w), _p(j_w),
                                 _p(ws), ws.numel(), s), "pds_kmeans_step")
    _lib.check(L.pds_kmeans_step_noalloc(plan.handle, _p(vals), _p(idx), n, K, _p(centers), _p(out_s), _p(a_s),
                                         _p(j_s), s), "pds_kmeans_step_noalloc")
    torch.cuda.synchronize()
    return (out_w.cpu().numpy(), a_w.cpu().numpy(), float(j_w.item())), \
           (out_s.cpu().numpy(), a_s.cpu().numpy(), float(j_s.item()))


@pytest.mark.parametrize("prec,p,m,K,n1,n2", [
    (pds.PDS_F32, 1024, 51, 10, 200000, 70001),   # cooperative FP32 path
    (pds.PDS_F32, 2048, 205, 40, 50000, 9999),    # FP32, K > 32
    (pds.PDS_F64, 256, 26, 5, 40000, 1234),       # FP64 plan
])
def test_noalloc_matches_workspace_call(prec, p, m, K, n1, n2):
    dt = np.float64 if prec == pds.PDS_F64 else np.float32
    plan = pds.Plan(p, m, seed=0, prec=prec)
    for n in (n1, n2):
        print(f"noalloc kmeans_step: prec={prec} p={p} m={m} K={K} n={n}", flush=True)
        d = synth.random_compressed(n, p, m, seed=n, dtype=dt, K=K)
        vals = torch.from_numpy(d["vals"]).cuda()
        idx = torch.from_numpy(d["idx"].view(np.int16)).cuda()
        centers = torch.from_numpy(d["centers"]).cuda()
        (cw, aw, jw), (cs, as_, js) = _both(plan, vals, idx, centers)
        assert np.array_equal(aw, as_), "assignments differ between the two entry points"
        assert aw.min() >= 0 and aw.max() < K
        # every K-means sum is fixed point: the same bits from both entry points
        assert np.array_equal(cw, cs), "centers differ between the two entry points"
        assert jw == js


def test_noalloc_rejects_sizes_beyond_its_scratch():
    L = pds.lib()
    plan = pds.Plan(4096, 410, seed=0, prec=pds.PDS_F32)
    n, K = 1 << 22, 50
    need = plan.workspace_size(pds.PDS_OP_KMEANS, n, K)
    assert need > _lib.PDS_NOALLOC_SCRATCH_BYTES
    fake = ctypes.c_void_p(256)  # never dereferenced: the call fails on the host first
    st = L.pds_kmeans_step_noalloc(plan.handle, fake, fake, n, K, fake, ctypes.c_void_p(512), fake, fake,
                                   ctypes.c_void_p(0))
    assert st == _lib.PDS_E_WORKSPACE
    assert b"scratch" in L.pds_last_error()
