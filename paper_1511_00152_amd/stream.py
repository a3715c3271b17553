"""Out-of-core estimation from rows held in host memory.

The paper's out-of-core runs load the data in chunks (about 1 GB each) and
compress every chunk once, so the full matrix is never resident.  Here the
chunks of a host array (through two pinned staging buffers unless the array
is itself in pinned memory) are copied to two device buffers on a stream of
their own, so the copy of chunk c + 1 runs while chunk c is compressed and
accumulated on the caller's stream; events order the reuse of each buffer.
Every chunk is compressed with its global row offset (sample i keeps the
coordinates of sample i whatever the chunking), then fed to the streaming
covariance and sample-mean accumulators, so the results equal a single call
on all rows up to the order of FP64 additions.  Rows narrower than the plan's
p are zero-padded on the device.
"""
from . import CovarianceAccumulator, Plan, compress, sample_mean


def stream_estimates(plan: Plan, X_host, chunk_rows: int, covariance: bool = True, mean: bool = True):
    """Covariance estimate C_n (p x p FP64) and sample-mean estimate (p FP64,
    preconditioned domain) of the rows of X_host (numpy array or CPU tensor,
    n x p_data, p_data <= plan.p, the plan's element type), streamed in chunks
    of chunk_rows rows.  Returns (C or None, mean or None)."""
    import numpy as np
    import torch

    if isinstance(X_host, np.ndarray):
        X_host = torch.from_numpy(X_host)
    if X_host.device.type != "cpu" or X_host.dim() != 2:
        raise ValueError("X_host must be a 2-D host array")
    if X_host.dtype != plan.dtype:
        raise TypeError(f"X_host dtype {X_host.dtype} does not match plan dtype {plan.dtype}")
    n, pd = X_host.shape
    if pd > plan.p or n < 1 or chunk_rows < 1:
        raise ValueError("need 1 <= n, 1 <= chunk_rows and columns <= plan.p")
    dev = torch.device("cuda", torch.cuda.current_device())
    chunk_rows = min(int(chunk_rows), n)
    # rows already in pinned memory go to the device directly; others are
    # staged through two pinned buffers first
    direct = X_host.is_pinned() and X_host.is_contiguous()
    pinned = [None, None] if direct else [torch.empty((chunk_rows, pd), dtype=plan.dtype, pin_memory=True)
                                          for _ in range(2)]
    staged = [torch.empty((chunk_rows, pd), dtype=plan.dtype, device=dev) for _ in range(2)]
    copied = [torch.cuda.Event() for _ in range(2)]
    consumed = [torch.cuda.Event() for _ in range(2)]
    compute = torch.cuda.current_stream()
    copier = torch.cuda.Stream()
    vals = torch.empty((chunk_rows, plan.m), dtype=plan.dtype, device=dev)
    idx = torch.empty((chunk_rows, plan.m), dtype=torch.int16, device=dev)
    cov = CovarianceAccumulator(plan) if covariance else None
    macc = torch.zeros(plan.p, dtype=torch.float64, device=dev) if mean else None
    used = [False, False]
    for c, a in enumerate(range(0, n, chunk_rows)):
        b = min(a + chunk_rows, n)
        rows = b - a
        s = c % 2
        if direct:
            src = X_host[a:b]
        else:
            if used[s]:
                copied[s].synchronize()  # the previous copy out of pinned[s] is done
            pinned[s][:rows].copy_(X_host[a:b])
            src = pinned[s][:rows]
        with torch.cuda.stream(copier):
            if used[s]:
                copier.wait_event(consumed[s])  # staged[s] is free again
            staged[s][:rows].copy_(src, non_blocking=True)
            copied[s].record(copier)
        used[s] = True
        compute.wait_event(copied[s])
        v, i = compress(plan, staged[s][:rows], i0=a, vals=vals[:rows], idx=idx[:rows])
        if cov is not None:
            cov.add(v, i)
        if macc is not None:
            sample_mean(plan, v, i, acc=macc, finalize=False)
        consumed[s].record(compute)
    C = cov.finalize() if cov is not None else None
    mu = sample_mean(plan, vals[:0], idx[:0], acc=macc, finalize=True, n_total=n) if mean else None
    torch.cuda.synchronize()
    return C, mu
