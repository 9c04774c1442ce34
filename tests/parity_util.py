"""Comparison helpers shared by the GPU parity tests (no method arithmetic).

Norm-wise errors alone are dominated by the rows of surrogate-face cells, which carry the
penalty sigma = gamma p^2 / h and the extrapolated point values; an error confined to the
other rows could hide under them.  The row-scaled check bounds every entry by the size of
the terms that make it up:

    |v_i - vref_i| <= tol * (|A| |u|)_i ,

with |A| the entry-wise absolute value of the oracle's assembled matrix.  A row whose terms
are all zero must then be exactly zero.
"""

import numpy as np


def rel(a, b):
    """Relative 2-norm error ||a - b|| / ||b|| (0 when both are empty or zero)."""
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / nb) if nb > 0 else float(np.linalg.norm(a))


def rel_inf(a, b):
    """max_i |a_i - b_i| / max_i |b_i|."""
    nb = np.max(np.abs(b)) if b.size else 0.0
    return float(np.max(np.abs(a - b)) / nb) if nb > 0 else float(np.max(np.abs(a), initial=0.0))


def row_scaled_excess(v, vref, A, u, tol):
    """Largest ratio |v_i - vref_i| / (tol * (|A||u|)_i) over the rows (<= 1 passes), and the
    index where it occurs.  Rows with (|A||u|)_i = 0 must match exactly (ratio inf if not)."""
    scale = abs(A) @ np.abs(u)
    diff = np.abs(v - vref)
    with np.errstate(divide="ignore", invalid="ignore"):
        ratio = np.where(scale > 0, diff / (tol * scale), np.where(diff > 0, np.inf, 0.0))
    if ratio.size == 0:
        return 0.0, -1
    i = int(np.argmax(ratio))
    return float(ratio[i]), i


def sampled_rows(O, prob, u, dofs):
    """Rows `dofs` of the oracle's A u and of |A||u|, formed one row at a time from the local
    matrices (cell matrix, surrogate-face matrices, and for DG the interior-face blocks) of
    the cells that hold each DoF: the oracle at sizes where assembling all of A is too slow.
    Returns (v_rows, scale_rows)."""
    dofs = np.asarray(dofs, dtype=np.int64)
    want = {int(g): k for k, g in enumerate(dofs)}
    v = np.zeros(dofs.size)
    s = np.zeros(dofs.size)
    Ac = O.cell_matrix(prob)
    cd = prob.cell_dofs
    hit = np.isin(cd, dofs)
    cells = np.nonzero(hit.any(axis=1))[0]
    faces_of = {}
    for f, (c, _, _) in enumerate(prob.sbm_faces):
        faces_of.setdefault(int(c), []).append(f)
    for c in cells:
        loc = cd[c]
        uk = u[loc]
        mats = [Ac] + [O.sbm_face_matrix(prob, f) for f in faces_of.get(int(c), [])]
        for li in np.nonzero(hit[c])[0]:
            k = want[int(loc[li])]
            for M in mats:
                v[k] += M[li] @ uk
                s[k] += np.abs(M[li]) @ np.abs(uk)
    if prob.disc == "dg":
        ifc = prob.interior_faces
        for fi in np.nonzero(hit[ifc[:, 0]].any(axis=1) | hit[ifc[:, 1]].any(axis=1))[0]:
            ks = (int(ifc[fi, 0]), int(ifc[fi, 1]))
            blocks = O.dg_face_blocks(prob, fi)
            for ti in range(2):
                for li in np.nonzero(hit[ks[ti]])[0]:
                    k = want[int(cd[ks[ti], li])]
                    for tj in range(2):
                        row = blocks[(ti, tj)][li]
                        uk = u[cd[ks[tj]]]
                        v[k] += row @ uk
                        s[k] += np.abs(row) @ np.abs(uk)
    return v, s
