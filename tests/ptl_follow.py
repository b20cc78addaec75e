"""Check of an advance cycled at the practical time step limit without a
floor (Eqs. (ptl)-(ptl3) as printed, ptl_floor = 0) against the oracle.

A cycle that steps at the limit flattens the limiting pair (Eq. (ptl2) at
equality): afterwards the pair's difference u_k - u_nb is small against
the values it is taken from, so the next limit -du/dF carries the relative
rounding error of du amplified by kappa = (|u_k| + |u_nb|) / |du| (and of dF
by (|F_k| + |F_nb|) / |dF|); once du is at the rounding level, even whether
the pair constrains (du dF < 0) is decided by the last bits of each side's
field.  The cycle lengths, and with them the schedule, may then part
between the GPU and the oracle.  The check lets the oracle replay the GPU's
schedule (cycle lengths, stages per cycle) from the same initial field and
requires, cycle by cycle, that the GPU's cycle length is a decision Eq.
(ptl3) gives on that state within its conditioning: the decision taken from
a cell whose |F| is within 1e-12 of the largest (the oracle's own cell or
one tied with it), with all its constraining pairs or with its flattened
pairs (|u_k - u_nb| <= 1e-9 (|u_k| + |u_nb|)) left out, equal within
(1e-12 + 1e-13 kappa) plus the one-cycle granularity of the cycle count;
or, where a flattened pair exists, a cycle of negligible length (<= 1e-6
dt_E).  A stage count that differs must be the stage formula's for the
cycle length moved by 1e-12.  The replayed field must match the GPU's to
1e-12.
"""
import math

import numpy as np


def _pairs_at(u, F, m):
    """Eq. (ptl2) at cell m (flat index) with each face neighbour (periodic in
    phi, none across a pole or a radial boundary): a list of (-du/dF or None
    when the pair does not constrain, kappa, flattened)."""
    nc, nr, nt, np_ = F.shape
    c, i, j, k = np.unravel_index(m, F.shape)
    nbs = []
    if i > 0:
        nbs.append((c, i - 1, j, k))
    if i < nr - 1:
        nbs.append((c, i + 1, j, k))
    if j > 0:
        nbs.append((c, i, j - 1, k))
    if j < nt - 1:
        nbs.append((c, i, j + 1, k))
    nbs += [(c, i, j, (k - 1) % np_), (c, i, j, (k + 1) % np_)]
    out = []
    for nb in nbs:
        uk, un, Fk, Fn = u[c, i, j, k], u[nb], F[c, i, j, k], F[nb]
        du, dF = uk - un, Fk - Fn
        ok = du != 0.0 and dF != 0.0 and du * dF < 0.0
        us = abs(uk) + abs(un)
        kappa = (us / abs(du) if du else math.inf) + ((abs(Fk) + abs(Fn)) / abs(dF) if dF else math.inf)
        out.append((-du / dF if ok else None, kappa, abs(du) <= 1e-9 * us))
    return out


def limit_candidates(o, u):
    """The pairs of Eq. (ptl2) at the cell of largest |F| (lowest linear
    index on ties, first) and at every cell whose |F| is within 1e-12 of it."""
    F = o.apply(u)
    a = np.abs(F).ravel()
    m0 = int(np.argmax(a))
    ms = [m0] + [int(m) for m in np.flatnonzero(a >= a[m0] * (1.0 - 1e-12)) if m != m0]
    return [_pairs_at(u, F, m) for m in ms]


def _limit(pairs):
    """(limit, kappa of the pair that sets it)."""
    valid = [p for p in pairs if p[0] is not None]
    if not valid:
        return math.inf, 0.0
    p = min(valid, key=lambda p: p[0])
    return p[0], p[1]


def _decision(t_rem, lim):
    nreq = math.ceil(t_rem / lim)
    return t_rem if nreq <= 1 else t_rem / nreq


def replay_unfloored(om, o, u0, dt, st, sts="rkl2", log=print):
    """The oracle replaying the GPU's unfloored schedule st from u0, with
    the checks above; returns (field, number of cycles not decided as the
    oracle's own decision to 1e-12)."""
    dtE = o.dt_explicit()
    u = np.array(u0, dtype=np.float64, copy=True)
    t_rem = dt
    ill = 0
    dts, ns = np.asarray(st["dt_cycle"], dtype=np.float64), np.asarray(st["per_cycle"])
    assert len(dts) == st["cycles"] == len(ns)
    for cyc, (dtc, n) in enumerate(zip(dts, ns)):
        cells = limit_candidates(o, u)
        lim0, _ = _limit(cells[0])
        assert lim0 == o.ptl(u)[0]
        dto = _decision(t_rem, lim0)
        if abs(dtc - dto) > 1e-12 * dto:
            options = []
            for c in cells:
                options.append(_limit(c))
                options.append(_limit([p for p in c if not p[2]]))
            agree = False
            for lim, kappa in options:
                if not math.isfinite(lim):
                    continue
                d = _decision(t_rem, lim)
                tol = (1e-12 + 1e-13 * kappa) * d + (d * d / t_rem if d < t_rem else 0.0)
                agree = agree or abs(dtc - d) <= tol
            flats = [p for c in cells for p in c if p[2]]
            log(f"  cycle {cyc}: {dtc / dtE!r} dt_E against the oracle's {dto / dtE!r}; tied cells "
                f"{len(cells) - 1}; conditioning of the oracle's limit {_limit(cells[0])[1]:.2e}; "
                f"flattened pairs {len(flats)}")
            assert agree or (flats and dtc <= 1e-6 * dtE), cyc
            ill += 1
        own = om.sts_stages(sts, dtc / dtE)
        if own != int(n):
            near = {om.sts_stages(sts, dtc / dtE * (1.0 + e)) for e in (-1e-12, 1e-12)}
            log(f"  cycle {cyc}: stage count {int(n)} against the oracle's {own} "
                f"(counts within 1e-12: {near})")
            assert int(n) in near, (cyc, own, int(n))
        u, _ = o.advance_sts(u, dtc, 1, sts, s_override=int(n))
        t_rem -= dtc
    return u, ill
