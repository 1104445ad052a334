"""Helpers shared by the GPU tests: device buffers, oracle comparisons, case logging."""
import sys

import numpy as np

import oracle


def log(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


def dev_u64(n):
    import torch
    return torch.empty(max(n, 1), dtype=torch.int64, device="cuda")


def dev_f64(n):
    import torch
    return torch.empty(max(n, 1), dtype=torch.float64, device="cuda")


def host_u64(t, n=None):
    import torch
    torch.cuda.synchronize()
    a = t.detach().cpu().numpy().view(np.uint64)
    return a if n is None else a[:n]


def host_f64(t, n=None):
    import torch
    torch.cuda.synchronize()
    a = t.detach().cpu().numpy()
    return a if n is None else a[:n]


def assert_same(c_gpu, r_gpu, c_ref, r_ref, what=""):
    """Bit-exact comparison of c and r (r compared as raw IEEE bits)."""
    if c_ref is not None:
        bad = np.nonzero(c_gpu != c_ref)[0]
        assert bad.size == 0, "%s: c mismatch at %s (gpu %s ref %s)" % (
            what, bad[:5], c_gpu[bad[:5]], c_ref[bad[:5]])
    if r_ref is not None:
        gb, rb = r_gpu.view(np.uint64), r_ref.view(np.uint64)
        bad = np.nonzero(gb != rb)[0]
        assert bad.size == 0, "%s: r mismatch at %s (gpu %s ref %s)" % (
            what, bad[:5], r_gpu[bad[:5]], r_ref[bad[:5]])


def oracle_gen(inst, k0, count):
    return oracle.generate(inst.p, inst.q, inst.e, inst.m0, inst.s0, k0, count)


def oracle_stats(inst, k0, count):
    return oracle.consume(inst.p, inst.q, inst.e, inst.m0, inst.s0, k0, count)
