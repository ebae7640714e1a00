"""Helpers for the GPU tests: run the HIP join through the C ABI binding and
bring the pair set back as a sorted (P, 2) int32 numpy array."""
import numpy as np
import torch

from paper_1908_11740_amd import sj


def to_dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def sort_pairs(p):
    p = np.asarray(p, dtype=np.int32).reshape(-1, 2)
    return p[np.lexsort((p[:, 1], p[:, 0]))]


def gpu_join(R, S, K, split_tau=0, flags=0, domain=None, count=False):
    Rd, Sd = to_dev(R), to_dev(S)
    PR = sj.partition(Rd, K, split_tau=split_tau, flags=flags, domain=domain)
    PS = sj.partition(Sd, K, split_tau=split_tau, flags=flags, domain=domain)
    if count:
        n = sj.join_count(PR, PS)
        PR.free()
        PS.free()
        return n
    out = sj.join(PR, PS)
    torch.cuda.synchronize()
    res = sort_pairs(out.cpu().numpy())
    PR.free()
    PS.free()
    return res
