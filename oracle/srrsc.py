"""Structured low-rank compression of Cauchy-like blocks (SRRSC).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

A Cauchy-like block A_ij = u_i v_j / (d_i - w_j) is compressed from its
generators alone (section "SRRSC low-rank approximation"):

* The k-th Schur complement A^(k) is Cauchy-like with the same nodes and
  generators updated one pivot at a time (Theorem 1, eq. UU / VV2):
      u^(k)(l) = u^(k-1)(l) (d_l - d_k) / (d_l - w_k)
      v^(k)(l) = v^(k-1)(l) (w_l - w_k) / (w_l - d_k)
  where (d_k, w_k) are the row node and column node of the k-th pivot.
  (The theorem's displacement equation carries an index garble, D_k where
  D_{k+1} is defined; the recursions above are what it states.)
* Pivots are chosen by complete pivoting on |A^(k)| (the paper allows it),
  ties broken by the smallest (row, column) position.  Elimination stops when
  every entry of the Schur complement is at most ``tol`` in magnitude; the
  pivot columns form the skeleton set T (eq. sid).
* The interpolation matrix Z = A11^{-1} A12 is Cauchy-like with row nodes the
  skeleton column nodes and column nodes the remaining column nodes
  (Theorem 2), with row generator (eq. yk)
      y(i) = prod_{j != i} (d_j - w_i)/(w_j - w_i) * (d_i - w_i) / v^(0)(i)
  over the pivots, and column generator v^(k) of the remaining columns.
  Entries (eq. geneZ, read against Theorem 2's displacement equation since
  the printed formula mixes u and y):  Z_ij = y(i) v^(k)(j) / (w_i - w_j).
* A P ~= A(:, T) [I Z]  (eq. sid); the neglected part is exactly A^(k), so
  every entry of the approximation is within ``tol`` of A.

Column nodes are given as w_j = wbase_j + woff_j (for a merge, the pole of
the root's origin plus its offset) so that node differences are formed
without cancellation: d_i - w_j = (d_i - wbase_j) - woff_j and
w_a - w_b = (wbase_a - wbase_b) + (woff_a - woff_b).
"""

import numpy as np


class CauchyBlock:
    """Generators of A_ij = u_i v_j / (d_i - w_j)."""

    def __init__(self, u, v, d, wbase, woff):
        self.u = np.asarray(u, dtype=np.float64)
        self.v = np.asarray(v, dtype=np.float64)
        self.d = np.asarray(d, dtype=np.float64)
        self.wbase = np.asarray(wbase, dtype=np.float64)
        self.woff = np.asarray(woff, dtype=np.float64)

    def d_minus_w(self, rows, cols):
        return (self.d[rows][:, None] - self.wbase[cols][None, :]) - self.woff[cols][None, :]

    def w_minus_w(self, a, b):
        return (self.wbase[a][:, None] - self.wbase[b][None, :]) + (
            self.woff[a][:, None] - self.woff[b][None, :])

    def dense(self):
        r = np.arange(self.u.shape[0])
        c = np.arange(self.v.shape[0])
        return self.u[:, None] * self.v[None, :] / self.d_minus_w(r, c)


def compress(blk, tol, max_rank=None):
    """Complete-pivoting SRRSC of one Cauchy-like block.

    Returns a dict with the pivot rows ``prow``, skeleton columns ``pcol``
    (both in pivot order), the remaining columns ``rest``, the row generator
    ``y`` of Z (length r) and the column generator ``vk`` of Z (length
    len(rest)).
    """
    m, n = blk.u.shape[0], blk.v.shape[0]
    max_rank = min(m, n) if max_rank is None else max_rank
    rows = np.arange(m)
    cols = np.arange(n)
    u = blk.u.copy()
    v = blk.v.copy()
    prow, pcol = [], []
    while len(prow) < max_rank and rows.size and cols.size:
        S = u[rows][:, None] * v[cols][None, :] / blk.d_minus_w(rows, cols)
        a = np.abs(S)
        flat = int(np.argmax(a))          # first maximum in row-major order
        i, j = divmod(flat, cols.size)
        if a[i, j] <= tol:
            break
        pr, pc = int(rows[i]), int(cols[j])
        prow.append(pr)
        pcol.append(pc)
        rows = np.delete(rows, i)
        cols = np.delete(cols, j)
        # Theorem 1: update the generators of the next Schur complement.
        pr_a = np.array([pr])
        pc_a = np.array([pc])
        if rows.size:
            dd = blk.d[rows] - blk.d[pr]
            dw = blk.d_minus_w(rows, pc_a)[:, 0]
            u[rows] = u[rows] * dd / dw
        if cols.size:
            ww = blk.w_minus_w(cols, pc_a)[:, 0]
            wd = -blk.d_minus_w(pr_a, cols)[0, :]      # w_l - d_k
            v[cols] = v[cols] * ww / wd
    prow = np.array(prow, dtype=np.int64)
    pcol = np.array(pcol, dtype=np.int64)
    r = prow.size
    # Theorem 2, eq. yk: row generator of Z over the pivots.
    y = np.empty(r)
    if r:
        dw = blk.d_minus_w(prow, pcol)        # (d_{prow a} - w_{pcol b})
        ww = blk.w_minus_w(pcol, pcol)        # (w_a - w_b)
        for a_ in range(r):
            others = [b for b in range(r) if b != a_]
            num = dw[others, a_]              # d_j - w_i, j != i
            den = -ww[a_, others]             # w_j - w_i
            y[a_] = np.prod(num / den) * dw[a_, a_] / blk.v[pcol[a_]]
    return {"prow": prow, "pcol": pcol, "rest": cols.copy(), "y": y,
            "vk": v[cols].copy(), "rank": r}


def interpolation_matrix(blk, comp):
    """Z (r x len(rest)) from the generators, eq. geneZ as read above."""
    pcol, rest = comp["pcol"], comp["rest"]
    if pcol.size == 0 or rest.size == 0:
        return np.zeros((pcol.size, rest.size))
    return comp["y"][:, None] * comp["vk"][None, :] / blk.w_minus_w(pcol, rest)


def approximate(blk, comp):
    """Dense A(:, T)[I Z] P^T: the block as the low-rank path sees it."""
    m, n = blk.u.shape[0], blk.v.shape[0]
    out = np.zeros((m, n))
    pcol, rest = comp["pcol"], comp["rest"]
    if pcol.size == 0:
        return out
    rows = np.arange(m)
    skel = blk.u[:, None] * blk.v[pcol][None, :] / blk.d_minus_w(rows, pcol)
    out[:, pcol] = skel
    if rest.size:
        out[:, rest] = skel @ interpolation_matrix(blk, comp)
    return out


def merge_block(Dbar, org, tau, zhat, s, rows, cols):
    """The (rows, cols) block of a merge's U as a CauchyBlock.

    With ``org is None`` the column nodes are tau itself (general Cauchy
    generators, as in the paper's Examples 0 and 1).
    """
    if org is None:
        return CauchyBlock(zhat[rows], s[cols], Dbar[rows], tau[cols],
                           np.zeros(cols.size))
    return CauchyBlock(zhat[rows], s[cols], Dbar[rows], Dbar[org[cols]],
                       tau[cols])


def lowrank_cauchy(Dbar, org, tau, zhat, s, tol, b):
    """Dense U with every off-diagonal b x b block replaced by its SRRSC form.

    Blocks are contiguous index ranges of the sorted order (block data
    distribution; section "Storage form affects the off-diagonally low-rank
    property").  Diagonal blocks are kept exact (PSMMA step 3(b): a block whose
    row and column index sets meet is treated as full rank).  Returns
    (U_approx, ranks) with ranks[I, J] the skeleton size of block (I, J)
    (-1 on the diagonal).
    """
    K = Dbar.shape[0]
    nb = (K + b - 1) // b
    U = np.empty((K, tau.shape[0]))
    ranks = -np.ones((nb, nb), dtype=np.int64)
    for I in range(nb):
        ri = np.arange(I * b, min(K, (I + 1) * b))
        for J in range(nb):
            cj = np.arange(J * b, min(K, (J + 1) * b))
            blk = merge_block(Dbar, org, tau, zhat, s, ri, cj)
            if I == J:
                U[np.ix_(ri, cj)] = blk.dense()
            else:
                comp = compress(blk, tol)
                U[np.ix_(ri, cj)] = approximate(blk, comp)
                ranks[I, J] = comp["rank"]
    return U, ranks
