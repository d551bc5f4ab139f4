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


def outer_masks(batch):
    """Per block, a boolean array of its stored shape marking the outer ghost
    points: ghost points in a direction whose neighbour entry is -1."""
    out = []
    for b, blk in enumerate(batch.blocks):
        ng = blk.ng
        k, j, i = np.meshgrid(np.arange(blk.nz + 2 * ng) - ng, np.arange(blk.ny + 2 * ng) - ng,
                              np.arange(blk.nx + 2 * ng) - ng, indexing="ij")
        ox = np.where(i < 0, -1, np.where(i >= blk.nx, 1, 0))
        oy = np.where(j < 0, -1, np.where(j >= blk.ny, 1, 0))
        oz = np.where(k < 0, -1, np.where(k >= blk.nz, 1, 0))
        ghost = (ox != 0) | (oy != 0) | (oz != 0)
        d = (oz + 1) * 9 + (oy + 1) * 3 + (ox + 1)
        out.append(ghost & (np.asarray(batch.neighbours)[b][d] < 0))
    return out


def compare(batch, gpu, o64, o80, nfields=W.NF, base=None, blocks=None, names=None,
            rel_floor=1e-3, gate=1e-12, masks=None):
    """Rows (field, e_gpu, e_oracle64, tol, max|o|) over the interior points,
    or, with `masks` (per block, a boolean array of the stored shape), over
    the marked points."""
    names = names or (W.FIELDS if nfields == W.NF else W.CONSTRAINTS)
    blocks = range(len(batch.blocks)) if blocks is None else blocks
    if masks is None:
        pick = lambda arr, b, f: batch.interior(arr, b, f, nfields).ravel()
    else:
        pick = lambda arr, b, f: batch.view(arr, b, f, nfields)[masks[b]]
    rows = []
    for f in range(nfields):
        g = np.concatenate([pick(gpu, b, f) for b in blocks])
        c = np.concatenate([pick(o64, b, f) for b in blocks])
        o = np.concatenate([pick(o80, b, f) for b in blocks])
        allow = 0.0
        if base is not None:
            z = np.concatenate([pick(base, b, f) for b in blocks])
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
