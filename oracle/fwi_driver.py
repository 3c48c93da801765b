"""Oracle: the inversion driver around the misfit gradient -- frequency
continuation over overlapping bands, stochastic subsampling of the sources,
and a box-constrained limited-memory BFGS -- in float64 (TEST
INFRASTRUCTURE; never imported by the GPU library).

Paper: the 2D inversion example (frequency bands of 4 with an overlap of 2,
20 iterations of a box-constrained L-BFGS per band, each band warm-started
from the previous one, the source/frequency mask selecting the band) and the
stochastic inversion section (minimise the average of f_i over a subset I_k
of the sources drawn uniformly at random, subject to m_LB <= m <= m_UB;
r_sub * ceil(N_s / p) iterations per subproblem; the approximate minimiser
warm-starts the next draw, T draws; |I_k| grows by a fixed amount when a line
search fails; the 3D example clamps the water layer to the true model, i.e.
per-point bounds).  The paper calls an external box-constrained quasi-Newton
code without describing its steps; the projected L-BFGS below is the
reading taken here, written out in full:

At x with gradient g the free set F leaves out variables at a bound whose
gradient points out of the box (x <= lo with g > 0, or x >= hi with g < 0).
The direction d is -H g restricted to F: the two-loop recursion over the
stored pairs (s_i, y_i), every vector restricted to F, rho_i = 1 / (y_i.s_i)
(0 when that is 0), initial scaling gamma = s.y / y.y of the newest pair (1
when y.y = 0); d = 0 off F.  With no stored pair, or when g.d >= 0, d =
-g_F * step0 / max|g_F|.  The subproblem stops when max|g_F| <= gtol times
its value at the subproblem's starting point (or is 0).  Backtracking: x_t = clamp(x + t d, lo, hi) for t =
1, 1/2, ... (at most max_ls trials), accepted when f(x_t) <= f(x) + c1
g.(x_t - x); every trial evaluates f and g.  The pair (x_t - x, g_t - g) is
stored when s.y > 1e-10 |s| |y| (the oldest dropped beyond `memory`).  A
failed line search ends the subproblem (the iterate stays) and grows the subset for the next
draw.  Every subproblem starts with an empty memory.  The subset size p
persists across draws and bands; p >= N_s selects every source.

Source subsets: a partial Fisher-Yates shuffle of 0..N_s-1 whose swap
partner at step i is i + (u mod (N_s - i)), u the next output of SplitMix64
(the published 64-bit generator of Steele, Lea and Flood: output k of seed s
mixes z = s + (k + 1) * 0x9E3779B97F4A7C15 with z ^= z >> 30, z *=
0xBF58476D1CE4E5B9, z ^= z >> 27, z *= 0x94D049BB133111EB, z ^= z >> 31);
the counter runs over the whole inversion; the subset is sorted ascending.
A draw of every source consumes no numbers.
"""
from __future__ import annotations

import numpy as np

from . import fwi
from . import operators as ops

MASK64 = (1 << 64) - 1


def splitmix64(seed, counter):
    """Output number `counter` (0, 1, ...) of SplitMix64 started at `seed`."""
    z = (seed + (counter + 1) * 0x9E3779B97F4A7C15) & MASK64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK64
    return z ^ (z >> 31)


class Draws:
    def __init__(self, seed):
        self.seed = seed & MASK64
        self.counter = 0

    def next(self):
        v = splitmix64(self.seed, self.counter)
        self.counter += 1
        return v


def draw_subset(draws: Draws, n, p):
    """p distinct indices of 0..n-1, uniformly at random, sorted (all n, and
    no numbers drawn, when p >= n)."""
    if p >= n:
        return list(range(n))
    a = list(range(n))
    for i in range(p):
        j = i + draws.next() % (n - i)
        a[i], a[j] = a[j], a[i]
    return sorted(a[:p])


def bands(nfreq, size, overlap):
    """Frequency bands [b, min(b + size, nfreq)) for b = 0, size - overlap,
    ..., up to the first band that reaches the last frequency."""
    if size < 1 or not 0 <= overlap < size:
        raise ValueError("band size >= 1 and 0 <= overlap < size")
    step = size - overlap
    out, b = [], 0
    while True:
        out.append(list(range(b, min(b + size, nfreq))))
        if b + size >= nfreq:
            return out
        b += step


def projected_lbfgs(fg, x, lo, hi, iters, memory, step0, c1=1e-4, max_ls=10, gtol=1e-6, log=None):
    """The box-constrained L-BFGS of the module docstring.  fg(x) -> (f, g).
    Returns (x, failed); failed is True when a line search failed (x is then
    the last accepted iterate).  log (a list) receives one dict per
    iteration: f at the iterate, f at the accepted (or last) trial, the number
    of trials, whether it was accepted and the accepted t."""
    x = np.clip(np.asarray(x, dtype=np.float64), lo, hi)
    f, g = fg(x)
    S, Y = [], []
    g0max = None
    for it in range(iters):
        free = ~(((x <= lo) & (g > 0)) | ((x >= hi) & (g < 0)))
        gF = np.where(free, g, 0.0)
        gmax = float(np.abs(gF).max())
        g0max = gmax if g0max is None else g0max
        if gmax == 0.0 or gmax <= gtol * g0max:
            return x, False
        d = None
        if S:
            q = gF.copy()
            hist = []
            for s, y in zip(reversed(S), reversed(Y)):
                sF, yF = np.where(free, s, 0.0), np.where(free, y, 0.0)
                ys = float(np.vdot(yF, sF))
                rho = 1.0 / ys if ys != 0.0 else 0.0
                a = rho * float(np.vdot(sF, q))
                q = q - a * yF
                hist.append((a, rho, sF, yF))
            sN, yN = np.where(free, S[-1], 0.0), np.where(free, Y[-1], 0.0)
            yy = float(np.vdot(yN, yN))
            r = (float(np.vdot(sN, yN)) / yy if yy > 0.0 else 1.0) * q
            for a, rho, sF, yF in reversed(hist):
                r = r + (a - rho * float(np.vdot(yF, r))) * sF
            d = -r
            if float(np.vdot(g, d)) >= 0.0:
                d = None
        if d is None:
            d = -gF * (step0 / gmax)
        t, accepted = 1.0, False
        for trial in range(1, max_ls + 1):
            xt = np.clip(x + t * d, lo, hi)
            ft, gt = fg(xt)
            if ft <= f + c1 * float(np.vdot(g, xt - x)):
                accepted = True
                break
            t *= 0.5
        if log is not None:
            log.append(dict(iter=it, f=f, f_new=ft, trials=trial, accepted=accepted, step=t, pgmax=gmax))
        if not accepted:
            return x, True
        s, y = xt - x, gt - g
        if float(np.vdot(s, y)) > 1e-10 * float(np.linalg.norm(s)) * float(np.linalg.norm(y)):
            S.append(s)
            Y.append(y)
            if len(S) > memory:
                S.pop(0)
                Y.pop(0)
        x, f, g = xt, ft, gt
    return x, False


def iterations(r_sub, nsrc, p):
    """Iteration limit of a subproblem on p of nsrc sources: r_sub ceil(N_s / p)."""
    return r_sub * -(-nsrc // min(p, nsrc))


def default_step0(lo, hi):
    """Max-norm length of a steepest-descent trial: 5 % of the range the
    bounds span, max(hi) - min(lo)."""
    return 0.05 * (float(np.max(hi)) - float(np.min(lo)))


def fwi_invert(g: ops.Grid, m0, lo, hi, omegas, src, rec, d, amp=None, band_size=4, band_overlap=2,
               r_sub=20, memory=5, batch=0, subproblems=1, batch_increase=1, seed=0, c1=1e-4,
               max_ls=10, gtol=1e-6, step0=None, stencil="7pt", w27=None, objective=None, log=None):
    """Frequency continuation x stochastic subproblems x projected L-BFGS on
    the averaged least-squares misfit over on-node sources and receivers
    (exact solves).  d: [nfreq][nsrc][nrec]; lo, hi: scalars or arrays of
    the model's shape.  objective(x, mask) -> (f, g) replaces the misfit
    (tests).  log receives one dict per subproblem (band, draw, the sources,
    its iteration limit, the per-iteration records, failed).  Returns the
    final model."""
    nf, ns = len(omegas), len(src)
    step0 = default_step0(lo, hi) if step0 is None else step0
    draws = Draws(seed)
    m = np.clip(np.asarray(m0, dtype=np.float64), lo, hi)
    p = ns if batch <= 0 else min(batch, ns)
    for bi, band in enumerate(bands(nf, band_size, band_overlap)):
        for t in range(subproblems):
            sel = draw_subset(draws, ns, p)
            mask = np.zeros((nf, ns), bool)
            for fi in band:
                mask[fi, sel] = True

            def fg(x, mask=mask):
                if objective is not None:
                    return objective(x, mask)
                f, grad, _, _ = fwi.misfit_gradient_pairs(g, x, omegas, src, rec, d, amp=amp, mask=mask,
                                                          renormalise=True, stencil=stencil, w27=w27)
                return f, grad

            steps = []
            nit = iterations(r_sub, ns, p)
            m, failed = projected_lbfgs(fg, m, lo, hi, nit, memory, step0, c1, max_ls, gtol, steps)
            if log is not None:
                log.append(dict(band=bi, draw=t, sources=sel, iters=nit, steps=steps, failed=failed))
            if failed:
                p = min(ns, p + batch_increase)
    return m
