"""NumPy brute force (test infrastructure): a second, independent FP64
implementation of the greedy that re-solves Phi_S from scratch with a library
solver at every iteration, for tiny and small inputs only.

* ``wendland``         Eq. (2)
* ``gcb_brute``        Algorithm 1 with a from-scratch dense solve every
                       iteration (the literal reading of its "compute Phi for
                       S; solve" steps) instead of the RC recurrence
* ``traditional_greedy`` the Rendall-Allen greedy of Section 1: errors at all
                       boundary nodes every iteration, append the global worst
"""
from __future__ import annotations

import numpy as np


def wendland(eta: np.ndarray) -> np.ndarray:
    eta = np.asarray(eta, dtype=np.float64)
    a = np.clip(1.0 - eta, 0.0, None)
    return a ** 4 * (4.0 * eta + 1.0)


def dist(a: np.ndarray, b: np.ndarray) -> np.ndarray:
    d = a[:, None, :] - b[None, :, :]
    return np.sqrt((d * d).sum(axis=2))


def rbf_matrix(a: np.ndarray, b: np.ndarray, radius: float) -> np.ndarray:
    return wendland(dist(a, b) / radius)


def solve_weights(xyz_S: np.ndarray, disp_S: np.ndarray, radius: float) -> np.ndarray:
    """W = Phi_S^-1 Delta_S by a library LU solve (Eqs. 4-5 restricted to S)."""
    return np.linalg.solve(rbf_matrix(xyz_S, xyz_S, radius), disp_S)


def start_nodes(xyz: np.ndarray, disp: np.ndarray) -> list[int]:
    """Farthest-point starting rule, ties to the lowest index (np.argmax)."""
    n0 = int(np.argmax((disp ** 2).sum(axis=1)))
    d0 = ((xyz - xyz[n0]) ** 2).sum(axis=1)
    n1 = int(np.argmax(d0))
    d1 = ((xyz - xyz[n1]) ** 2).sum(axis=1)
    n2 = int(np.argmax(np.minimum(d0, d1)))
    return [n0, n1, n2]


def gcb_brute(xyz, disp, radius, group_of, m, tol_abs, nc_max=None, init=None, warm=None, per_iter=1):
    """Algorithm 1 by brute force.  Returns (S, log) with log entries
    (k, group, node, E, appended).  warm: a kept support set to start from
    (no iteration if it already meets tol_abs at every node, else k starts
    at len(warm)).  per_iter > 1: the several-nodes-per-iteration variant
    (block form of the peak-selection idea cited in Section 1): every node of
    the group whose error exceeds tol_abs is ranked by (error descending, index
    ascending) and the first per_iter of them (fewer if |S| would pass nc_max)
    are appended; `appended` in the log is then their count."""
    if per_iter > 1:
        return _block_brute(xyz, disp, radius, group_of, m, tol_abs, nc_max, init, per_iter)
    xyz = np.asarray(xyz, np.float64)
    disp = np.asarray(disp, np.float64)
    nb = xyz.shape[0]
    nc_max = nb if nc_max is None else nc_max
    log = []
    if warm is not None:
        S = [int(j) for j in warm]
        W = solve_weights(xyz[S], disp[S], radius)
        F = rbf_matrix(xyz, xyz[S], radius) @ W
        if np.sqrt(((F - disp) ** 2).sum(axis=1)).max() <= tol_abs:
            return S, log
        k, quiet = len(S), 0
    else:
        S = list(start_nodes(xyz, disp) if init is None else init)
        k, quiet = 3, 0
    while True:
        g = k % m
        W = solve_weights(xyz[S], disp[S], radius)
        cand = [j for j in range(nb) if group_of[j] == g and j not in S]
        if cand:
            F = rbf_matrix(xyz[cand], xyz[S], radius) @ W
            e = np.sqrt(((F - disp[cand]) ** 2).sum(axis=1))
            t = int(np.argmax(e))           # first maximum = lowest node index (cand ascending)
            E, n = float(e[t]), cand[t]
        else:
            E, n = 0.0, -1
        app = False
        stop = False
        if n >= 0 and E > tol_abs:
            if len(S) < nc_max:
                S.append(n)
                app = True
                quiet = 0
            else:
                stop = True
        else:
            quiet += 1
        log.append((k, g, n, E, app))
        k += 1
        if stop or quiet >= m:
            break
    return S, log


def _block_brute(xyz, disp, radius, group_of, m, tol_abs, nc_max, init, per_iter):
    xyz = np.asarray(xyz, np.float64)
    disp = np.asarray(disp, np.float64)
    nb = xyz.shape[0]
    nc_max = nb if nc_max is None else nc_max
    S = list(start_nodes(xyz, disp) if init is None else init)
    k, quiet, log = 3, 0, []
    while True:
        g = k % m
        W = solve_weights(xyz[S], disp[S], radius)
        cand = np.array([j for j in range(nb) if group_of[j] == g and j not in S], dtype=np.int64)
        E, n, take, stop = 0.0, -1, [], False
        if cand.size:
            F = rbf_matrix(xyz[cand], xyz[S], radius) @ W
            e = np.sqrt(((F - disp[cand]) ** 2).sum(axis=1))
            order = np.lexsort((cand, -e))          # error descending, then index ascending
            E, n = float(e[order[0]]), int(cand[order[0]])
            over = [int(cand[t]) for t in order if e[t] > tol_abs]
            if over:
                room = nc_max - len(S)
                if room <= 0:
                    stop = True
                take = over[: min(per_iter, max(room, 0))]
        S.extend(take)
        if take:
            quiet = 0
        elif not stop:
            quiet += 1
        log.append((k, g, n, E, len(take)))
        k += 1
        if stop or quiet >= m:
            break
    return S, log


def traditional_greedy(xyz, disp, radius, tol_abs, nc_max=None, init=None):
    """Rendall-Allen greedy: all-node errors each iteration, append the worst node."""
    xyz = np.asarray(xyz, np.float64)
    disp = np.asarray(disp, np.float64)
    nb = xyz.shape[0]
    nc_max = nb if nc_max is None else nc_max
    S = list(start_nodes(xyz, disp) if init is None else init)
    inS = np.zeros(nb, dtype=bool)
    inS[S] = True
    while True:
        W = solve_weights(xyz[S], disp[S], radius)
        F = rbf_matrix(xyz, xyz[S], radius) @ W
        e = np.sqrt(((F - disp) ** 2).sum(axis=1))
        e[inS] = -1.0
        n = int(np.argmax(e))
        if e[n] <= tol_abs or len(S) >= nc_max:
            return S
        S.append(n)
        inS[n] = True
