"""Helpers shared by the GPU parity tests."""
import numpy as np

import oracle
import paper_2004_04817_amd as gcb


def gpu_select(p, tol_abs=None, nc_max=None, m=None, init_idx=None, group_of=None, precision=gcb.GCB_PREC_FP64):
    tol = p.tol_abs if tol_abs is None else tol_abs
    ctx = gcb.Context(0)
    ctx.set_boundary(p.xyz, p.disp)
    ctx.set_params(p.radius, p.m if m is None else m, tol, nc_max=nc_max, seed=p.seed, precision=precision,
                   init_idx=init_idx)
    if group_of is not None:
        ctx.set_groups(group_of)
    info = ctx.select()
    S, W = ctx.get_support()
    log = ctx.get_log()
    return ctx, info, S, W, log


def oracle_select(p, tol_abs=None, nc_max=None, m=None, init_idx=None, group_of=None):
    tol = p.tol_abs if tol_abs is None else tol_abs
    return oracle.select(p.xyz, p.disp, p.radius, p.m if m is None else m, tol, nc_max=nc_max, seed=p.seed,
                         init_idx=init_idx, group_of=group_of, nthreads=0)


def first_divergence(a, b):
    n = min(len(a), len(b))
    d = np.flatnonzero(np.asarray(a[:n]) != np.asarray(b[:n]))
    return int(d[0]) if len(d) else (n if len(a) != len(b) else -1)
