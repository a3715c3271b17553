"""Batched form: many independent data sets (own p, m, K, seed each)
compressed in one persistent launch and clustered by T rounds of sparsified
K-means replayed from one captured HIP graph (pds_batch_* in include/pds.h).

    b = Batch([dict(X=X0, m=26, K=5, seed=0), dict(X=X1, m=51, K=10, seed=1)], T=20)
    b.compress(); b.init_centers(); b.kmeans()
    b.sets[0]["centers"], b.sets[0]["assign"], b.sets[0]["objective"]

Argument marshalling only; every step runs in libpds kernels.
"""
import ctypes

from . import _ptr, _stream
from ._lib import PdsBatchDesc, check, lib


class Batch:
    def __init__(self, sets, T, device="cuda"):
        import torch

        self.T = int(T)
        self.sets = []
        descs = (PdsBatchDesc * len(sets))()
        for i, s in enumerate(sets):
            X = s["X"]
            n, p = X.shape
            m, K = int(s["m"]), int(s["K"])
            if X.dtype != torch.float32 or X.stride(1) != 1:
                raise TypeError("X must be float32 with contiguous rows")
            e = dict(X=X, n=n, p=p, m=m, K=K, seed=int(s.get("seed", 0)),
                     vals=torch.empty((n, m), dtype=torch.float32, device=device),
                     idx=torch.empty((n, m), dtype=torch.int16, device=device),
                     centers=s.get("centers", torch.zeros((K, p), dtype=torch.float64, device=device)),
                     centers_alt=torch.empty((K, p), dtype=torch.float64, device=device),
                     assign=torch.empty(n, dtype=torch.int32, device=device),
                     objective=torch.zeros(max(self.T, 1), dtype=torch.float64, device=device))
            self.sets.append(e)
            d = descs[i]
            d.X, d.n, d.ldx, d.p, d.m, d.K, d.reserved, d.seed = (X.data_ptr(), n, X.stride(0), p, m, K, 0,
                                                                  e["seed"])
            d.vals, d.idx = e["vals"].data_ptr(), e["idx"].data_ptr()
            d.centers, d.centers_alt = e["centers"].data_ptr(), e["centers_alt"].data_ptr()
            d.assign, d.objective = e["assign"].data_ptr(), e["objective"].data_ptr()
        self._descs = descs
        h = ctypes.c_void_p()
        check(lib().pds_batch_create(ctypes.byref(h), descs, len(sets), self.T), "pds_batch_create")
        self._h = h
        b = ctypes.c_size_t(0)
        check(lib().pds_batch_workspace_size(h, ctypes.byref(b)), "pds_batch_workspace_size")
        self.ws = torch.empty(int(b.value), dtype=torch.uint8, device=device)
        check(lib().pds_batch_bind(h, _ptr(self.ws), self.ws.numel(), _stream()), "pds_batch_bind")

    def compress(self):
        check(lib().pds_batch_compress(self._h, _stream()), "pds_batch_compress")

    def init_centers(self):
        check(lib().pds_batch_init_centers(self._h, _stream()), "pds_batch_init_centers")

    def kmeans(self):
        check(lib().pds_batch_kmeans(self._h, _stream()), "pds_batch_kmeans")

    def autotune(self):
        check(lib().pds_batch_autotune(self._h, _stream()), "pds_batch_autotune")

    def info(self):
        buf = ctypes.create_string_buffer(1024)
        check(lib().pds_batch_info(self._h, buf, len(buf)), "pds_batch_info")
        return dict(kv.split("=") for kv in buf.value.decode().split())

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            lib().pds_batch_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
