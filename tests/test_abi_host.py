"""Host-side checks of the C ABI (no GPU): the library loads, exports every
entry point include/pds.h declares, validates arguments before touching the
device, and its host-computed sign diagonal equals the oracle's."""
import ctypes
import os
import re

import numpy as np
import pytest

import paper_1511_00152_amd as pds
from paper_1511_00152_amd import _lib
from oracle import ref

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "pds.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(pds_[a-z_0-9]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    L = pds.lib()
    names = declared_functions()
    assert len(names) >= 10
    for n in names:
        assert hasattr(L, n), n
    assert set(names) == set(_lib.EXPORTS)
    assert pds.lib().pds_version().startswith(b"pds")


def _plan_status(p, m, prec=pds.PDS_F32):
    h = ctypes.c_void_p()
    st = pds.lib().pds_plan_create(ctypes.byref(h), p, m, 0, prec)
    if st == 0:
        pds.lib().pds_plan_destroy(h)
    return st


@pytest.mark.parametrize("p,m,expect", [
    (256, 26, 0), (2, 1, 0), (2, 2, 0), (65536, 100, 0),
    (6, 3, _lib.PDS_E_UNSUPPORTED), (1, 1, _lib.PDS_E_UNSUPPORTED), (131072, 5, _lib.PDS_E_UNSUPPORTED),
    (0, 0, _lib.PDS_E_UNSUPPORTED), (784, 40, _lib.PDS_E_UNSUPPORTED),
    (256, 0, _lib.PDS_E_M), (256, 257, _lib.PDS_E_M), (256, -1, _lib.PDS_E_M),
])
def test_plan_validation(p, m, expect):
    assert _plan_status(p, m) == expect


def test_plan_rejects_unknown_precision_and_null_out():
    assert _plan_status(256, 26, prec=7) == _lib.PDS_E_ARG
    assert pds.lib().pds_plan_create(None, 256, 26, 0, 1) == _lib.PDS_E_ARG
    assert b"NULL" in pds.lib().pds_last_error()


@pytest.mark.parametrize("seed,p", [(0, 256), (0, 4096), (123456789, 1024), (2 ** 63 + 5, 65536), (3, 2)])
def test_host_signs_equal_oracle(seed, p):
    plan = pds.Plan(p, 1, seed=seed)
    assert np.array_equal(plan.signs(), ref.signs(seed, p))


def test_hot_calls_validate_before_device_work():
    L = pds.lib()
    plan = pds.Plan(256, 26, prec=pds.PDS_F32)
    h = plan.handle
    fake = ctypes.c_void_p(0x1000)
    null = ctypes.c_void_p(0)
    # compress
    assert L.pds_compress(None, fake, 4, 256, 0, fake, fake, null, 0, null) == _lib.PDS_E_ARG
    assert L.pds_compress(h, fake, -1, 256, 0, fake, fake, null, 0, null) == _lib.PDS_E_ARG
    assert L.pds_compress(h, null, 4, 256, 0, fake, fake, null, 0, null) == _lib.PDS_E_ARG
    assert L.pds_compress(h, fake, 4, 255, 0, fake, fake, null, 0, null) == _lib.PDS_E_ARG
    assert L.pds_compress(h, null, 0, 0, 0, null, null, null, 0, null) == _lib.PDS_OK  # n == 0 no-op
    # covariance
    plan1 = pds.Plan(256, 1, prec=pds.PDS_F32)
    assert L.pds_covariance(plan1.handle, fake, fake, 4, fake, 1, 4, fake, fake, 1 << 30, null) == _lib.PDS_E_M
    assert L.pds_covariance(h, fake, fake, 4, null, 0, 0, null, fake, 1 << 30, null) == _lib.PDS_E_ARG
    assert L.pds_covariance(h, null, fake, 4, fake, 0, 0, null, fake, 1 << 30, null) == _lib.PDS_E_ARG
    assert L.pds_covariance(h, fake, fake, 4, fake, 1, 0, fake, fake, 1 << 30, null) == _lib.PDS_E_ARG
    assert L.pds_covariance(h, fake, fake, 4, fake, 1, 4, null, fake, 1 << 30, null) == _lib.PDS_E_ARG
    assert L.pds_covariance(h, null, null, 0, fake, 0, 0, null, null, 0, null) == _lib.PDS_OK
    # kmeans
    assert L.pds_kmeans_step(h, fake, fake, 4, 0, fake, fake, fake, fake, fake, 1 << 30, null) == _lib.PDS_E_ARG
    assert L.pds_kmeans_step(h, fake, fake, 4, 1025, fake, fake, fake, fake, fake, 1 << 30, null) == _lib.PDS_E_ARG
    assert L.pds_kmeans_step(h, fake, fake, 4, 3, fake, fake, null, fake, fake, 1 << 30, null) == _lib.PDS_E_ARG
    assert L.pds_kmeans_step(h, fake, fake, 4, 3, fake, fake, fake, fake, fake, 1 << 30, null) == _lib.PDS_E_ARG  # alias
    assert L.pds_kmeans_step(h, null, null, 0, 3, null, null, null, null, null, 0, null) == _lib.PDS_OK
    # kmeans without allocation: same argument checks, before any device query
    assert L.pds_kmeans_step_noalloc(None, fake, fake, 4, 3, fake, fake, fake, fake, null) == _lib.PDS_E_ARG
    assert L.pds_kmeans_step_noalloc(h, fake, fake, -1, 3, fake, fake, fake, fake, null) == _lib.PDS_E_ARG
    assert L.pds_kmeans_step_noalloc(h, fake, fake, 4, 0, fake, fake, fake, fake, null) == _lib.PDS_E_ARG
    assert L.pds_kmeans_step_noalloc(h, fake, fake, 4, 1025, fake, fake, fake, fake, null) == _lib.PDS_E_ARG
    assert L.pds_kmeans_step_noalloc(h, fake, fake, 4, 3, fake, fake, null, fake, null) == _lib.PDS_E_ARG
    assert L.pds_kmeans_step_noalloc(h, fake, fake, 4, 3, fake, fake, fake, fake, null) == _lib.PDS_E_ARG  # alias
    assert L.pds_kmeans_step_noalloc(h, null, null, 0, 3, null, null, null, null, null) == _lib.PDS_OK
    # several rounds in one call
    two = ctypes.c_void_p(0x2000)
    assert L.pds_kmeans_run(None, fake, fake, 4, 3, 2, fake, two, fake, fake, fake, 1 << 30, null) == _lib.PDS_E_ARG
    assert L.pds_kmeans_run(h, fake, fake, -1, 3, 2, fake, two, fake, fake, fake, 1 << 30, null) == _lib.PDS_E_ARG
    assert L.pds_kmeans_run(h, fake, fake, 4, 0, 2, fake, two, fake, fake, fake, 1 << 30, null) == _lib.PDS_E_ARG
    assert L.pds_kmeans_run(h, fake, fake, 4, 3, 0, fake, two, fake, fake, fake, 1 << 30, null) == _lib.PDS_E_ARG
    assert L.pds_kmeans_run(h, fake, fake, 4, 3, 2, fake, two, fake, null, fake, 1 << 30, null) == _lib.PDS_E_ARG
    assert L.pds_kmeans_run(h, fake, fake, 4, 3, 2, fake, fake, fake, fake, fake, 1 << 30, null) == _lib.PDS_E_ARG
    assert L.pds_kmeans_run(h, null, null, 0, 3, 2, null, null, null, null, null, 0, null) == _lib.PDS_OK
    assert plan.workspace_size(pds.PDS_OP_KMEANS_RUN, 1000, 5) > plan.workspace_size(pds.PDS_OP_KMEANS, 1000, 5)
    # unmix
    assert L.pds_unmix(h, fake, 0, ctypes.c_void_p(0x2000), null) == _lib.PDS_E_ARG
    assert L.pds_unmix(h, null, 2, fake, null) == _lib.PDS_E_ARG
    assert L.pds_unmix(h, fake, 2, fake, null) == _lib.PDS_E_ARG


def test_workspace_queries():
    plan = pds.Plan(4096, 410, prec=pds.PDS_SPLIT_BF16)
    assert plan.workspace_size(pds.PDS_OP_COMPRESS if hasattr(pds, "PDS_OP_COMPRESS") else 0, 1 << 20) == 0
    cov = plan.workspace_size(1, 1 << 20)
    # block offsets (17 per sample) + FP32 partial tiles
    assert cov >= (1 << 20) * 17 * 4
    assert plan.workspace_size(1, 0) == 0
    km = pds.Plan(1024, 51).workspace_size(2, 1 << 20, 10)
    assert km > 0
    b = ctypes.c_size_t()
    assert pds.lib().pds_workspace_size(plan.handle, 2, 10, 0, ctypes.byref(b)) == _lib.PDS_E_ARG
    assert pds.lib().pds_workspace_size(plan.handle, 9, 10, 1, ctypes.byref(b)) == _lib.PDS_E_ARG
    assert pds.lib().pds_covariance_acc_size(plan.handle, ctypes.byref(b)) == 0 and b.value == 4096 * 4096 * 8
    # huge p needs a compress workspace (transform staging outside LDS): the
    # row buffer fits in LDS up to p = 8192 in FP32 and 4096 in FP64
    assert pds.Plan(65536, 10).workspace_size(0, 1000) > 0
    for p, prec, zero in ((8192, pds.PDS_F32, True), (16384, pds.PDS_F32, False), (4096, pds.PDS_F64, True),
                          (8192, pds.PDS_F64, False), (8192, pds.PDS_SPLIT_BF16, True)):
        assert (pds.Plan(p, 10, prec=prec).workspace_size(0, 1000) == 0) == zero, (p, prec)


def test_estimator_calls_validate_before_device_work():
    """The sample-mean, seeding, best-of-R, padding and explained-variance
    calls reject bad arguments on the host (status codes, no device work)."""
    L = pds.lib()
    plan = pds.Plan(256, 26, prec=pds.PDS_F32)
    h = plan.handle
    fake = ctypes.c_void_p(0x1000)
    null = ctypes.c_void_p(0)
    # sample mean
    assert L.pds_sample_mean(h, fake, fake, -1, fake, 0, 0, null, fake, 1 << 30, null) == _lib.PDS_E_ARG
    assert L.pds_sample_mean(h, fake, fake, 4, null, 0, 0, null, fake, 1 << 30, null) == _lib.PDS_E_ARG
    assert L.pds_sample_mean(h, null, fake, 4, fake, 0, 0, null, fake, 1 << 30, null) == _lib.PDS_E_ARG
    assert L.pds_sample_mean(h, fake, fake, 4, fake, 1, 0, ctypes.c_void_p(0x2000), fake, 1 << 30, null) == \
        _lib.PDS_E_ARG  # finalize with n_total = 0
    assert L.pds_sample_mean(h, fake, fake, 4, fake, 1, 4, fake, fake, 1 << 30, null) == _lib.PDS_E_ARG  # alias
    assert L.pds_sample_mean(h, null, null, 0, fake, 0, 0, null, null, 0, null) == _lib.PDS_OK  # nothing to do
    # K-means++ and best of R
    assert L.pds_kmeanspp(h, fake, fake, 0, 3, 0, fake, null, fake, 1 << 30, null) == _lib.PDS_E_ARG
    assert L.pds_kmeanspp(h, fake, fake, 4, 0, 0, fake, null, fake, 1 << 30, null) == _lib.PDS_E_ARG
    assert L.pds_kmeanspp(h, fake, fake, 4, 3, -1, fake, null, fake, 1 << 30, null) == _lib.PDS_E_ARG
    assert L.pds_kmeanspp(h, fake, fake, 4, 3, 0, null, null, fake, 1 << 30, null) == _lib.PDS_E_ARG
    assert L.pds_kmeans_best(h, fake, fake, 4, 3, 0, 2, fake, fake, fake, fake, fake, 1 << 30, null) == _lib.PDS_E_ARG
    assert L.pds_kmeans_best(h, fake, fake, 4, 3, 2, 0, fake, fake, fake, fake, fake, 1 << 30, null) == _lib.PDS_E_ARG
    assert L.pds_kmeans_best(h, fake, fake, 4, 3, 2, 2, fake, fake, null, fake, fake, 1 << 30, null) == _lib.PDS_E_ARG
    # padding and explained variance
    assert L.pds_pad_rows(fake, pds.PDS_F32, 4, 10, 10, ctypes.c_void_p(0x2000), 8, null) == _lib.PDS_E_ARG
    assert L.pds_pad_rows(fake, pds.PDS_F32, 4, 10, 9, ctypes.c_void_p(0x2000), 16, null) == _lib.PDS_E_ARG
    assert L.pds_pad_rows(fake, pds.PDS_F32, 4, 10, 10, fake, 16, null) == _lib.PDS_E_ARG  # alias
    assert L.pds_pad_rows(fake, 7, 4, 10, 10, ctypes.c_void_p(0x2000), 16, null) == _lib.PDS_E_ARG
    assert L.pds_pad_rows(null, pds.PDS_F32, 0, 10, 10, null, 16, null) == _lib.PDS_OK
    ws = _lib.PDS_EXPLAINED_WS_BYTES
    assert L.pds_explained_variance(fake, 33, fake, pds.PDS_F32, 4, 8, 8, fake, fake, ws, null) == _lib.PDS_E_ARG
    assert L.pds_explained_variance(fake, 2, fake, pds.PDS_F32, 4, 8, 7, fake, fake, ws, null) == _lib.PDS_E_ARG
    assert L.pds_explained_variance(fake, 2, fake, pds.PDS_F32, 0, 8, 8, fake, fake, ws, null) == _lib.PDS_E_ARG
    assert L.pds_explained_variance(fake, 2, fake, pds.PDS_F32, 4, 8, 8, fake, fake, ws - 1, null) == \
        _lib.PDS_E_WORKSPACE


def test_estimator_workspace_queries():
    plan = pds.Plan(4096, 410, prec=pds.PDS_SPLIT_BF16)
    assert plan.workspace_size(_lib.PDS_OP_MEAN, 0) == 0
    mean = plan.workspace_size(_lib.PDS_OP_MEAN, 1 << 20)
    assert 0 < mean <= 1024 * 4096 * 8 * 2  # a few partial rows per CU, not per sample
    pp = pds.Plan(1024, 51).workspace_size(_lib.PDS_OP_KMEANSPP, 1 << 20)
    assert pp >= (1 << 20) * 8  # D^2 per sample
    km = pds.Plan(1024, 51).workspace_size(_lib.PDS_OP_KMEANS, 1 << 20, 10)
    best = pds.Plan(1024, 51).workspace_size(_lib.PDS_OP_KMEANS_BEST, 1 << 20, 10)
    assert best >= km + pp + 2 * 10 * 1024 * 8 + (1 << 20) * 4
    b = ctypes.c_size_t()
    assert pds.lib().pds_workspace_size(plan.handle, _lib.PDS_OP_KMEANS_BEST, 10, 0, ctypes.byref(b)) == _lib.PDS_E_ARG


def test_stream_estimates_validates_on_the_host():
    """The out-of-core helper rejects inputs it cannot stream before touching
    the device."""
    torch = pytest.importorskip("torch")
    from paper_1511_00152_amd.stream import stream_estimates

    plan = pds.Plan(256, 26, prec=pds.PDS_F32)
    with pytest.raises(TypeError):
        stream_estimates(plan, np.zeros((10, 256), dtype=np.float64), 4)  # FP64 rows for an FP32 plan
    with pytest.raises(ValueError):
        stream_estimates(plan, np.zeros((10, 300), dtype=np.float32), 4)  # wider than p
    with pytest.raises(ValueError):
        stream_estimates(plan, np.zeros((0, 256), dtype=np.float32), 4)  # no rows
    with pytest.raises(ValueError):
        stream_estimates(plan, np.zeros((10, 256), dtype=np.float32), 0)  # empty chunks
    with pytest.raises(ValueError):
        stream_estimates(plan, torch.zeros(10, dtype=torch.float32), 4)  # not 2-D


def _dct_status(p, m, prec=pds.PDS_F32):
    h = ctypes.c_void_p()
    st = pds.lib().pds_plan_create_dct(ctypes.byref(h), p, m, 0, prec)
    if st == 0:
        pds.lib().pds_plan_destroy(h)
    return st


@pytest.mark.parametrize("p,m,prec,expect", [
    (784, 40, pds.PDS_F32, 0), (784, 784, pds.PDS_F64, 0), (2, 1, pds.PDS_F32, 0), (7, 3, pds.PDS_SPLIT_BF16, 0),
    (8192, 100, pds.PDS_F32, 0), (1024, 51, pds.PDS_F32, 0),
    (8193, 10, pds.PDS_F32, _lib.PDS_E_UNSUPPORTED), (1, 1, pds.PDS_F32, _lib.PDS_E_UNSUPPORTED),
    (784, 0, pds.PDS_F32, _lib.PDS_E_M), (784, 785, pds.PDS_F32, _lib.PDS_E_M), (784, 40, 9, _lib.PDS_E_ARG),
])
def test_dct_plan_validation(p, m, prec, expect):
    assert _dct_status(p, m, prec) == expect


def test_dct_plan_queries():
    """A DCT plan of any p (Sec. III's fast orthonormal transforms; Sec. VII's
    p = 784): its transform reads back, its signs and compress workspace (the
    FFT form's two p-point complex FP64 tables when p = 2^a 3^b 5^c 7^d <= 2048,
    else the dense form's p x p FP64 table), and a covariance accumulator over
    the next power of two; the m-selector calls refuse it."""
    L = pds.lib()
    plan = pds.Plan(784, 40, seed=5, transform=pds.PDS_TRANSFORM_DCT)
    t = ctypes.c_int32(-1)
    assert L.pds_plan_transform(plan.handle, ctypes.byref(t)) == 0 and t.value == pds.PDS_TRANSFORM_DCT
    assert L.pds_plan_transform(pds.Plan(256, 26).handle, ctypes.byref(t)) == 0 and t.value == 0
    assert L.pds_plan_transform(None, ctypes.byref(t)) == _lib.PDS_E_ARG
    assert L.pds_plan_transform(plan.handle, None) == _lib.PDS_E_ARG
    assert np.array_equal(plan.signs(), ref.signs(5, 784))
    assert plan.workspace_size(pds.PDS_OP_COMPRESS, 1000) == 2 * 784 * 16 + 256
    for q, fast in ((2, True), (1000, True), (2048, True), (4096, False), (129, False), (11, False), (2058, False)):
        w = pds.Plan(q, 1, transform=pds.PDS_TRANSFORM_DCT).workspace_size(pds.PDS_OP_COMPRESS, 10)
        assert w == (2 * q * 16 + 256 if fast else q * q * 8), q
    b = ctypes.c_size_t()
    assert L.pds_covariance_acc_size(plan.handle, ctypes.byref(b)) == 0 and b.value == 1024 * 1024 * 8
    assert plan.pg == 1024
    assert pds.Plan(1024, 51, transform=pds.PDS_TRANSFORM_DCT).pg == 1024
    assert plan.workspace_size(pds.PDS_OP_COVARIANCE, 1000) == pds.Plan(1024, 40).workspace_size(
        pds.PDS_OP_COVARIANCE, 1000)
    assert plan.workspace_size(pds.PDS_OP_KMEANS, 1000, 10) > 0
    sel = pds.Plan(784, 784, transform=pds.PDS_TRANSFORM_DCT)
    out = ctypes.c_int32()
    fake = ctypes.c_void_p(0x1000)
    assert L.pds_msel_label(sel.handle, fake, 10, 784, 0.1, ctypes.cast(ctypes.byref(out), ctypes.c_void_p), None,
                            fake, 1 << 30, None) == _lib.PDS_E_UNSUPPORTED


def test_gram_form_choice():
    """The automatic choice: FP32 plans take the sparse form at the workloads'
    small m/p (their dense tiles run on the slower FP32 matrix cores), split
    plans keep the BF16 matrix-core tiles at these sizes, every plan keeps the
    dense form when every coordinate is kept, FP64 plans stay dense."""
    assert pds.Plan(4096, 410, prec=pds.PDS_SPLIT_BF16).gram_form(1 << 20) == pds.PDS_GRAM_DENSE
    assert pds.Plan(4096, 410, prec=pds.PDS_F32).gram_form(1 << 20) == pds.PDS_GRAM_SPARSE
    assert pds.Plan(1024, 51, prec=pds.PDS_F32).gram_form(1 << 20) == pds.PDS_GRAM_SPARSE
    assert pds.Plan(1024, 1024, prec=pds.PDS_SPLIT_BF16).gram_form(1 << 20) == pds.PDS_GRAM_DENSE
    assert pds.Plan(1024, 1024, prec=pds.PDS_F32).gram_form(1 << 20) == pds.PDS_GRAM_DENSE
    assert pds.Plan(256, 26, prec=pds.PDS_F64).gram_form(2000) == pds.PDS_GRAM_DENSE
    assert pds.Plan(256, 26, prec=pds.PDS_F32, gram=pds.PDS_GRAM_DENSE).gram_form(2000) == pds.PDS_GRAM_DENSE
    b = ctypes.c_int32(0)
    L = pds.lib()
    plan = pds.Plan(256, 26, prec=pds.PDS_F64)
    assert L.pds_plan_set_gram(plan.handle, pds.PDS_GRAM_SPARSE) == _lib.PDS_E_UNSUPPORTED
    assert L.pds_plan_set_gram(plan.handle, 7) == _lib.PDS_E_ARG
    assert L.pds_plan_set_gram(None, 1) == _lib.PDS_E_ARG
    assert L.pds_plan_gram(plan.handle, -1, ctypes.byref(b)) == _lib.PDS_E_ARG
    assert L.pds_plan_gram(plan.handle, 10, None) == _lib.PDS_E_ARG
    # the two forms size their workspaces differently
    sp = pds.Plan(4096, 410, prec=pds.PDS_F32, gram=pds.PDS_GRAM_SPARSE).workspace_size(1, 1 << 20)
    de = pds.Plan(4096, 410, prec=pds.PDS_F32, gram=pds.PDS_GRAM_DENSE).workspace_size(1, 1 << 20)
    assert sp > 0 and de > 0 and sp != de
