"""Parity metric between the GPU path and the oracle (test helper).

Per field f and interior point p, with the extended-precision oracle o as
reference (the same oracle source computed in x87 extended precision):

    e(p) = |g(p) - o(p)| / max(|o(p)|, tau_f),   tau_f = 1e-3 * max_p |o_f|

The gate is  max_p e <= tol_f = max(1e-12, 8 * max_p e_oracle),  where
e_oracle is the same error of the FP64 oracle against o.  On fields whose
value is a near-cancellation of much larger terms (Theta on constraint-
satisfying data, At on the star metric) the FP64 oracle itself is only
good to a few 1e-12; there the GPU must be within 8x of the oracle's own
rounding error, elsewhere within 1e-12.  Why 8: the two evaluation orders
put each term of the longest sums (32 terms) through between 5 and 31
roundings, so their random-like rounding errors have spreads within a
factor (31/5)^(1/2) = 2.5 of each other, and the maximum over many points
moves that ratio by some 20 %; 8 is the power of two above twice 2.5 x 1.2.
Fields that are exactly zero in the oracle must be exactly zero on the GPU.

State outputs (a stage or a step) are compared through their increments
(state minus a base state), since states near 1 would make the comparison
vacuous.  The stage combination rounds up to six times at the magnitude of
the state on the GPU (two fused steps for u1, four for u0'), half an ulp
each, and the extended oracle once when it stores double: 3.5 units in the
last place (ulp), so for increments the error first has 4 ulp of the
stored state value subtracted:
    e(p) = max(|g - o| - 4 ulp(|x(p)|), 0) / max(|o|, tau_f).
"""
import numpy as np

from paper_2311_04989_amd import workloads as W


def compare(batch, gpu, o64, o80, nfields=W.NF, base=None, blocks=None, names=None,
            rel_floor=1e-3, gate=1e-12):
    names = names or (W.FIELDS if nfields == W.NF else W.CONSTRAINTS)
    blocks = range(len(batch.blocks)) if blocks is None else blocks
    rows = []
    for f in range(nfields):
        g = np.concatenate([batch.interior(gpu, b, f, nfields).ravel() for b in blocks])
        c = np.concatenate([batch.interior(o64, b, f, nfields).ravel() for b in blocks])
        o = np.concatenate([batch.interior(o80, b, f, nfields).ravel() for b in blocks])
        allow = 0.0
        if base is not None:
            z = np.concatenate([batch.interior(base, b, f, nfields).ravel() for b in blocks])
            allow = 4.0 * np.spacing(np.abs(o))
            g, c, o = g - z, c - z, o - z
        m = np.abs(o).max()
        if m == 0.0:
            rows.append((names[f], float(np.abs(g).max()), 0.0, 0.0, m))
            continue
        tau = rel_floor * m
        den = np.maximum(np.abs(o), tau)
        eg = float((np.maximum(np.abs(g - o) - allow, 0.0) / den).max())
        ec = float((np.maximum(np.abs(c - o) - allow, 0.0) / den).max())
        rows.append((names[f], eg, ec, max(gate, 8.0 * ec), m))
    return rows


# (case, worst e_gpu, worst e_fp64_oracle, worst e_gpu / tol) of every
# comparison made in this process; printed at the end of the test session
SUMMARY = []


def assert_parity(rows, label=""):
    case = label.split("\n")[0]
    graded = [(eg, ec, eg / tol) for _, eg, ec, tol, m in rows if m != 0.0]
    if graded:
        SUMMARY.append((case, max(g[0] for g in graded), max(g[1] for g in graded),
                        max(g[2] for g in graded)))
    bad = []
    for name, eg, ec, tol, m in rows:
        if m == 0.0:
            if eg != 0.0:
                bad.append(f"{name}: oracle exactly 0, GPU max |g| = {eg:.3e}")
        elif not eg <= tol:
            bad.append(f"{name}: e_gpu={eg:.3e} > tol={tol:.3e} (e_fp64_oracle={ec:.3e})")
    assert not bad, label + "\n" + "\n".join(bad)


def report(rows):
    return "\n".join(f"  {n:6s} e_gpu={eg:.2e} e_oracle64={ec:.2e} tol={tol:.2e} max|o|={m:.2e}"
                     for n, eg, ec, tol, m in rows)
