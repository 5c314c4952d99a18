"""Shared checks for the parity tests (tolerances and neighbour validity)."""
import math

import numpy as np


def fp64_tol(m: int) -> float:
    """Profile tolerance of the FP64 path: 1e-9 * 2 sqrt(m)."""
    return 1e-9 * 2.0 * math.sqrt(m)


def mixed_tol(m: int) -> float:
    """Profile tolerance of the mixed-precision paths: 1e-3 * 2 sqrt(m)."""
    return 1e-3 * 2.0 * math.sqrt(m)


def profile_close(P_gpu, P_ora, m: int, tol: float):
    """Element-wise: |dP| <= tol, or |P_gpu^2 - P_ora^2| <= 2 sqrt(m) tol.

    The squared form is the reading used near P = 0, where any correlation based
    evaluation loses digits (dP ~ sqrt(2 m drho)).  Infinite entries must agree.
    Returns (ok_mask, max_abs_err).
    """
    P_gpu = np.asarray(P_gpu, np.float64)
    P_ora = np.asarray(P_ora, np.float64)
    inf_g, inf_o = ~np.isfinite(P_gpu), ~np.isfinite(P_ora)
    ok = inf_g == inf_o
    fin = ~inf_g & ~inf_o
    with np.errstate(invalid="ignore"):
        d = np.abs(P_gpu - P_ora)
        d2 = np.abs(P_gpu ** 2 - P_ora ** 2)
    ok_f = (d <= tol) | (d2 <= 2.0 * math.sqrt(m) * tol)
    ok = ok & np.where(fin, ok_f, True)
    err = float(np.max(np.where(fin, d, 0.0))) if fin.any() else 0.0
    return ok, err


def check_neighbours(c_oracle, r, m, excl, rows, I_gpu, P_ora, tol):
    """Every reported neighbour is admissible and attains the oracle's NN distance."""
    rows = np.asarray(rows, np.int64)
    I_gpu = np.asarray(I_gpu, np.int64)
    fin = np.isfinite(P_ora)
    assert np.all(I_gpu[~fin] == -1), "rows without admissible partner must report -1"
    rr, ii = rows[fin], I_gpu[fin]
    assert np.all(np.abs(ii - rr) >= excl), "reported neighbour inside the exclusion zone"
    assert np.all((ii >= 0) & (ii < len(r) - m + 1))
    dd = c_oracle.pair_dist(r, m, rr, ii)
    ok, err = profile_close(dd, P_ora[fin], m, tol)
    bad = np.nonzero(~ok)[0]
    assert ok.all(), f"neighbour distance differs from the NN distance at rows {rr[bad[:5]]}: err {err}"


def discords_equivalent(gpu_list, ora_list, A_ora, m, tol):
    """Top-K lists agree: identical, or (near ties) each GPU pick is a valid
    eps-greedy pick on the oracle's combined profile.  Returns number of near-tie cases."""
    if [i for i, _, _ in gpu_list] == [i for i, _, _ in ora_list]:
        return 0
    alive = np.isfinite(A_ora)
    n_sub = len(A_ora)
    ties = 0
    for (i, g, s), (io, go, so) in zip(gpu_list, ora_list):
        best = float(np.max(np.where(alive, A_ora, -np.inf)))
        assert alive[i] and A_ora[i] >= best - 2 * tol, f"pick {i} is not a near-maximum ({A_ora[i]} vs {best})"
        if i != io:
            ties += 1
        alive[max(0, i - m + 1):min(n_sub, i + m)] = False
    return ties


def certified_top(c_oracle, R_np, m, excl, P_gpu, I_gpu, top_k):
    """Exact greedy top-K without a full oracle profile.

    U_g[i] = d(i, I_gpu[g, i]) is an upper bound of the exact P_g[i].  Rows are
    taken in descending max_g U; their exact profiles are computed until every
    greedy pick on exact values beats the largest bound of the rows not yet
    computed.  Returns (top list, A_exact dict, U matrix).
    """
    k, n_sub = P_gpu.shape
    rows = np.arange(n_sub)
    U = np.stack([c_oracle.pair_dist(R_np[g], m, rows, I_gpu[g]) for g in range(k)])
    U = np.where(I_gpu >= 0, U, -np.inf)
    AU = U.max(axis=0)
    order = np.argsort(-AU, kind="stable")
    exact = {}
    batch = 64
    pos = 0
    while True:
        new = order[pos:pos + batch]
        pos += len(new)
        Pn = np.stack([c_oracle.profile(R_np[g], m, excl, rows=new)[0] for g in range(k)])
        for q, i in enumerate(new):
            col = Pn[:, q]
            col = np.where(np.isfinite(col), col, -np.inf)
            exact[int(i)] = (float(col.max()), int(np.argmax(col)))
        tau_rows = order[pos:]
        alive = np.ones(n_sub, bool)
        picks = []
        certified = True
        for _ in range(top_k):
            cand = [(v, i) for i, (v, g) in exact.items() if alive[i] and v > -np.inf]
            rest = tau_rows[alive[tau_rows]]
            tau = AU[rest].max() if rest.size else -np.inf
            if not cand:
                # every computed row is masked: uncomputed live rows may still hold picks
                certified = not (tau > -np.inf)
                break
            v, i = max(cand, key=lambda t: (t[0], -t[1]))
            if tau >= v:
                certified = False
                break
            picks.append((i, exact[i][1], v))
            alive[max(0, i - m + 1):min(n_sub, i + m)] = False
        if certified or pos >= n_sub:
            return picks, exact, U
