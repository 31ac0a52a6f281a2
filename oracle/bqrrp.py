"""Plain FP64 CPU oracle of blocked randomized QR with column pivoting (BQRRP).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports, links or calls
this module: only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may use it.  It shares no code with the
HIP library; the two meet only in the seeded inputs built by ``workloads``.

It is deliberately slow and literal: NumPy vectors, explicit loops over the
sequential steps, one library primitive (a matmul, a triangular solve) per
step where a step *is* that primitive.  Every function names the passage of
the paper (arXiv 2507.00976, "Anatomy of High-Performance Column-Pivoted QR
Decomposition") it follows.  Indices are 0-based, as in the paper (Sec. 1.3).

Where the paper is silent or ambiguous, the reading taken is stated inline
at the step it shapes.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np
from scipy.linalg import solve_triangular

# status codes (same meaning as the C ABI's, defined independently here)
OK = 0
ERR_NONFINITE = 3

_M0 = np.uint64(0xD2511F53)
_M1 = np.uint64(0xCD9E8D57)
_W0 = np.uint32(0x9E3779B9)
_W1 = np.uint32(0xBB67AE85)
_MASK32 = np.uint64(0xFFFFFFFF)


# --------------------------------------------------------------------------
# Sketching operator (Alg. 1 sampling step; Sec. 3 "Initial sketching
# details"; Sec. 2 remark on using randomness once).
# --------------------------------------------------------------------------
def philox4x32_10(c0, c1, c2, c3, key):
    """Philox4x32 with 10 rounds (Salmon, Moraes, Dror, Shaw, SC'11).

    Each round multiplies counter words 0 and 2 by the two Philox multipliers,
    and forms the next counter from the high/low product halves, the other two
    counter words and the key; the key is advanced by the two Weyl constants
    between rounds.  Arguments are uint32 arrays (broadcastable), ``key`` a
    pair of uint32.  Returns the four output words.
    """
    c0, c1, c2, c3 = (np.asarray(x, dtype=np.uint32) for x in (c0, c1, c2, c3))
    k0 = np.uint32(key[0])
    k1 = np.uint32(key[1])
    with np.errstate(over="ignore"):
        for r in range(10):
            if r:
                k0 = np.uint32((int(k0) + int(_W0)) & 0xFFFFFFFF)
                k1 = np.uint32((int(k1) + int(_W1)) & 0xFFFFFFFF)
            p0 = _M0 * c0.astype(np.uint64)
            p1 = _M1 * c2.astype(np.uint64)
            hi0 = (p0 >> np.uint64(32)).astype(np.uint32)
            lo0 = (p0 & _MASK32).astype(np.uint32)
            hi1 = (p1 >> np.uint64(32)).astype(np.uint32)
            lo1 = (p1 & _MASK32).astype(np.uint32)
            c0, c1, c2, c3 = hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0
    return c0, c1, c2, c3


def seed_key(seed: int):
    return (seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF)


def gaussian_pairs(rows: np.ndarray, pair: int, seed: int, stream: int = 0):
    """Two N(0,1) values per (row, pair): Box-Muller on one Philox block.

    counter = (row, pair, stream, 0), key = (seed lo, seed hi).
    u1 = (2*(w >> 12) + 1) * 2^-53 in (0, 1) from words 0,1 (w = x1*2^32 + x0),
    u2 = (w' >> 11) * 2^-53 in [0, 1) from words 2,3,
    g0 = sqrt(-2 ln u1) cos(2 pi u2),  g1 = sqrt(-2 ln u1) sin(2 pi u2).
    """
    rows = np.asarray(rows, dtype=np.uint64)
    x0, x1, x2, x3 = philox4x32_10(rows & _MASK32, np.uint32(pair), np.uint32(stream), np.uint32(0),
                                   seed_key(seed))
    w01 = (x1.astype(np.uint64) << np.uint64(32)) | x0.astype(np.uint64)
    w23 = (x3.astype(np.uint64) << np.uint64(32)) | x2.astype(np.uint64)
    u1 = ((w01 >> np.uint64(12)).astype(np.float64) * 2.0 + 1.0) * 2.0 ** -53
    u2 = (w23 >> np.uint64(11)).astype(np.float64) * 2.0 ** -53
    rad = np.sqrt(-2.0 * np.log(u1))
    ang = (2.0 * math.pi) * u2
    return rad * np.cos(ang), rad * np.sin(ang)


def sketch_operator(d: int, m: int, seed: int) -> np.ndarray:
    """S in R^{d x m} with i.i.d. N(0,1) entries (Sec. 3: "S in R^{d x m}";
    the d-by-n wording of Alg. 1 is read as d-by-m since S multiplies M from
    the left).  Rows 2p and 2p+1 come from the Philox block (j, p, 0, 0) for
    matrix row j; an odd last row keeps only the cosine half.  S for a smaller
    d is the leading block of S for a larger d (prefix property)."""
    s = np.empty((d, m), dtype=np.float64)
    j = np.arange(m)
    for p in range((d + 1) // 2):
        g0, g1 = gaussian_pairs(j, p, seed)
        s[2 * p] = g0
        if 2 * p + 1 < d:
            s[2 * p + 1] = g1
    return s


def to_bf16(x: np.ndarray) -> np.ndarray:
    """FP64 -> FP32 -> BF16 (both round-to-nearest-even), returned as FP32."""
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    rnd = ((u >> np.uint64(16)) & np.uint64(1)) + np.uint64(0x7FFF)
    u = ((u + rnd) >> np.uint64(16)) << np.uint64(16)
    return u.astype(np.uint32).view(np.float32)


def sketch(a: np.ndarray, d: int, seed: int, precision: str = "f64") -> np.ndarray:
    """M^sk = S M (Alg. 1 sketching step).  ``precision="bf16"``: both operands
    rounded to BF16, products accumulated in FP32, result stored as FP64."""
    s = sketch_operator(d, a.shape[0], seed)
    if precision == "f64":
        return s @ a
    if precision == "bf16":
        return (to_bf16(s) @ to_bf16(a)).astype(np.float64)
    raise ValueError(precision)


# --------------------------------------------------------------------------
# qrcp_wide by LU (Alg. 2): GETRF on the transposed sketch, pivot format
# conversion, column permutation, GEQRF of the permuted sketch.
# --------------------------------------------------------------------------
def getrf_pivots(x: np.ndarray, steps: int | None = None):
    """Row-pivoted LU (GETRF semantics) of x (r x c), unblocked right-looking,
    over the first ``steps`` columns (all min(r, c) by default).

    Step j picks p = argmax_{t >= j} |x(t, j)| (ties -> smallest t, as IDAMAX),
    swaps rows j and p, and, if the pivot is nonzero, scales the column below
    it by the pivot and subtracts the rank-1 update from the trailing block.
    Returns (ipiv, margins): ipiv[j] = p (0-based, LAPACK swap format) and the
    relative gap between the best and second-best |candidate| at each step
    (1.0 when there is a single candidate), used to decide when pivot identity
    between two implementations is a fair requirement.
    """
    x = np.array(x, dtype=np.float64, copy=True)
    r, c = x.shape
    steps = min(r, c) if steps is None else min(r, c, steps)
    ipiv = np.empty(steps, dtype=np.int64)
    margins = np.ones(steps)
    for j in range(steps):
        col = np.abs(x[j:, j])
        p = j + int(np.argmax(col))
        if col.size > 1 and col[p - j] > 0:
            second = np.max(np.delete(col, p - j))
            margins[j] = (col[p - j] - second) / col[p - j]
        elif col.size > 1:
            margins[j] = 0.0
        ipiv[j] = p
        if p != j:
            x[[j, p], :] = x[[p, j], :]
        if x[j, j] != 0.0:
            x[j + 1:, j] /= x[j, j]
            x[j + 1:, j + 1:] -= np.outer(x[j + 1:, j], x[j, j + 1:])
    return ipiv, margins


def piv_transform(ipiv: np.ndarray, n: int) -> np.ndarray:
    """LU swap list -> permutation vector (Sec. 2.1 "Permutation formats"):
    start from the identity and, for each LU step j in order, exchange
    entries j and ipiv[j].  Result: column t of the permuted matrix was column
    J[t] of the input (0-based)."""
    jq = np.arange(n, dtype=np.int64)
    for j, p in enumerate(ipiv):
        jq[j], jq[p] = jq[p], jq[j]
    return jq


def larfg(alpha: float, x: np.ndarray):
    """Householder reflector in the LAPACK DLARFG convention:
    H [alpha; x] = [beta; 0], H = I - tau [1; v][1; v]^T,
    beta = -sign(alpha) * ||[alpha; x]|| with sign(0) = +1, tau = (beta-alpha)/beta,
    v = x / (alpha - beta); tau = 0 (H = I) when x = 0."""
    xx = float(x @ x) if x.size else 0.0
    if xx == 0.0:
        return alpha, np.zeros_like(x), 0.0
    beta = -math.copysign(math.sqrt(alpha * alpha + xx), alpha if alpha != 0.0 else 1.0)
    tau = (beta - alpha) / beta
    v = x / (alpha - beta)
    return beta, v, tau


def householder_qr(a: np.ndarray):
    """Unpivoted Householder QR (GEQRF semantics), column by column.

    Returns (R, V, tau): R upper trapezoidal (same shape as a, exact zeros
    below the diagonal), V unit lower trapezoidal (r x min(r,c)), tau."""
    a = np.array(a, dtype=np.float64, copy=True)
    r, c = a.shape
    kk = min(r, c)
    v_all = np.zeros((r, kk))
    tau = np.zeros(kk)
    for j in range(kk):
        beta, v, t = larfg(a[j, j], a[j + 1:, j])
        vv = np.concatenate(([1.0], v))
        if j + 1 < c and t != 0.0:
            w = vv @ a[j:, j + 1:]
            a[j:, j + 1:] -= t * np.outer(vv, w)
        a[j, j] = beta
        a[j + 1:, j] = 0.0
        v_all[j:, j] = vv
        tau[j] = t
    return np.triu(a), v_all, tau


def qrcp_wide_lu(msk: np.ndarray, steps: int | None = None):
    """Alg. 2: pivots of the wide sketch by GETRF on its transpose, the
    pivot-format conversion, the column permutation, then GEQRF.

    ``steps`` bounds the elimination steps by the rank the sketch can have:
    the sketch of a matrix with m_i rows has rank at most m_i, so beyond
    m_i steps the Schur complement of its transpose is zero in exact
    arithmetic and GETRF would pivot on rounding noise (only a wide matrix's
    last blocks have m_i < min(d, n_i)).

    Returns (Jsk, Rsk, ipiv, margins).  Rsk is min(d, n_i) x n_i upper
    trapezoidal; Q^sk is not needed by BQRRP and is discarded."""
    d, ni = msk.shape
    ipiv, margins = getrf_pivots(msk.T, steps)
    jsk = piv_transform(ipiv, ni)
    rsk, _, _ = householder_qr(msk[:, jsk])
    return jsk, rsk[: min(d, ni)], ipiv, margins


def qrcp_wide_geqp3(msk: np.ndarray, steps: int | None = None):
    """The alternative qrcp_wide: Businger-Golub column-norm pivoting of the
    sketch (GEQP3 semantics, norms recomputed exactly each step).  Only the
    first ``steps`` Householder steps pivot (the same rank bound as
    ``qrcp_wide_lu``); the rest keep the column order."""
    d, ni = msk.shape
    a = np.array(msk, dtype=np.float64, copy=True)
    jsk = np.arange(ni)
    psteps = min(d, ni) if steps is None else min(d, ni, steps)
    margins = np.ones(psteps)
    for j in range(min(d, ni)):
        p = j
        if j < psteps:
            norms = np.linalg.norm(a[j:, j:], axis=0)
            p = j + int(np.argmax(norms))
            # relative gap to the runner-up (as for the LU pivots)
            if norms.size > 1 and norms[p - j] > 0:
                margins[j] = (norms[p - j] - np.max(np.delete(norms, p - j))) / norms[p - j]
            elif norms.size > 1:
                margins[j] = 0.0
        if p != j:
            a[:, [j, p]] = a[:, [p, j]]
            jsk[[j, p]] = jsk[[p, j]]
        beta, v, t = larfg(a[j, j], a[j + 1:, j])
        vv = np.concatenate(([1.0], v))
        if j + 1 < ni and t != 0.0:
            w = vv @ a[j:, j + 1:]
            a[j:, j + 1:] -= t * np.outer(vv, w)
        a[j, j] = beta
        a[j + 1:, j] = 0.0
    return jsk, np.triu(a)[: min(d, ni)], None, margins


# --------------------------------------------------------------------------
# tri_rank (Sec. 2.2): the paper defers to a naive estimator; the reading
# used here is the leading run of diagonal entries that stay above
# tol * (largest column norm of the initial sketch).
# --------------------------------------------------------------------------
def tri_rank(rsk: np.ndarray, kmax: int, tol: float, ref: float) -> int:
    thr = tol * ref
    for t in range(kmax):
        v = abs(rsk[t, t])
        if not (v > thr):          # also catches NaN
            return t
    return kmax


# --------------------------------------------------------------------------
# qr_tall by preconditioned Cholesky QR + Householder reconstruction (Alg. 3,
# App. B background on Cholesky QR, Sec. 3 "Cholesky QR on a panel").
# --------------------------------------------------------------------------
def cholesky_upper(g: np.ndarray):
    """G = R^T R, R upper with positive diagonal, column by column.
    Returns (R, t) where t = number of columns factored before a
    non-positive (or NaN) pivot; R[:t, :t] is valid."""
    k = g.shape[0]
    r = np.zeros_like(g)
    for t in range(k):
        dd = g[t, t] - r[:t, t] @ r[:t, t]
        if not (dd > 0.0):
            return r, t
        r[t, t] = math.sqrt(dd)
        r[t, t + 1:] = (g[t, t + 1:] - r[:t, t] @ r[:t, t + 1:]) / r[t, t]
    return r, k


def cholqr(mpre: np.ndarray, passes: int = 1):
    """Cholesky QR (SYRK, POTRF, TRSM); ``passes=2`` repeats it on Q (CholQR2).
    Returns (Q, Rc, k_eff) with k_eff < k on a Cholesky breakdown."""
    k = mpre.shape[1]
    g = mpre.T @ mpre
    rc, t = cholesky_upper(g)
    if t < k:
        return None, rc[:t, :t], t
    q = solve_triangular(rc, mpre.T, trans="T", lower=False).T      # Q = M R^{-1}
    if passes == 2:
        g2 = q.T @ q
        r2, t2 = cholesky_upper(g2)
        if t2 < k:
            return None, rc[:t2, :t2], t2
        q = solve_triangular(r2, q.T, trans="T", lower=False).T
        rc = r2 @ rc
    return q, rc, k


def householder_reconstruct(q: np.ndarray):
    """Householder reconstruction of an explicit orthonormal Q (m x k), after
    Ballard et al. (BD2015, Alg. 5), as ORHR_COL: LU without pivoting of
    Q - [D; 0] with the sign D_j chosen on the fly as -sgn(current Q(j,j))
    (sgn(0) = +1).  Then Q - [D;0] = Y U, tau_j = -D_j U(j,j), and the first
    k columns of H = H_0 ... H_{k-1} equal Q diag(D).

    Returns (Y, tau, D, U): Y unit lower trapezoidal (m x k)."""
    w = np.array(q, dtype=np.float64, copy=True)
    m, k = w.shape
    dsig = np.empty(k)
    for j in range(k):
        dsig[j] = -1.0 if w[j, j] >= 0.0 else 1.0
        w[j, j] -= dsig[j]
        w[j + 1:, j] /= w[j, j]
        w[j + 1:, j + 1:] -= np.outer(w[j + 1:, j], w[j, j + 1:])
    u = np.triu(w[:k, :k])
    y = np.tril(w, -1)
    y[np.arange(k), np.arange(k)] = 1.0
    tau = -dsig * np.diag(u)
    return y, tau, dsig, u


def larft(y: np.ndarray, tau: np.ndarray) -> np.ndarray:
    """Upper triangular T of the compact WY form H_0...H_{k-1} = I - Y T Y^T
    (LARFT, forward, columnwise): T(j,j) = tau_j,
    T(0:j, j) = -tau_j T(0:j,0:j) (Y(:,0:j)^T Y(:,j))."""
    k = y.shape[1]
    t = np.zeros((k, k))
    for j in range(k):
        t[j, j] = tau[j]
        if j:
            t[:j, j] = -tau[j] * (t[:j, :j] @ (y[:, :j].T @ y[:, j]))
    return t


def apply_qt(y: np.ndarray, t: np.ndarray, c: np.ndarray) -> np.ndarray:
    """(I - Y T Y^T)^T C = C - Y T^T (Y^T C)  (ORMQR, left, transpose)."""
    w = y.T @ c
    w = t.T @ w
    return c - y @ w


# --------------------------------------------------------------------------
# The BQRRP loop (Alg. 1 with the in-place practical steps of Sec. 3).
# --------------------------------------------------------------------------
@dataclass
class BlockTrace:
    s: int
    k: int
    kmax: int
    ipiv: np.ndarray | None
    margins: np.ndarray
    jsk: np.ndarray
    msk_in: np.ndarray | None = None   # the sketch this block started from (if traced)


@dataclass
class Result:
    a: np.ndarray            # R above the diagonal, Householder vectors below
    jpiv: np.ndarray         # column t of AP is column jpiv[t] of A (0-based)
    tau: np.ndarray
    rank: int
    status: int = OK
    trace: list = field(default_factory=list)

    def min_margin(self) -> float:
        return min((float(np.min(b.margins)) for b in self.trace if b.margins.size), default=1.0)


def bqrrp(a: np.ndarray, b: int, gamma: float = 1.25, seed: int = 42, tol: float = 0.0,
          cholqr_passes: int = 1, qrcp_wide: str = "lu", sketch_precision: str = "f64",
          trailing_precision: str = "f64", msk: np.ndarray | None = None,
          trace_sketch: bool = False, max_blocks: int | None = None,
          qr_tall: str = "cholqr", max_rank: int | None = None) -> Result:
    """BQRRP (Alg. 1) with a choice of qrcp_wide (LU, Alg. 2, or GEQP3 on the
    sketch) and of qr_tall (preconditioned Cholesky QR + reconstruction,
    Alg. 3, or Householder QR of the panel, GEQRF; Sec. 2.3).

    Per block i (s = i b, n_i = n - s, m_i = m - s,
    k_max = min(b, n_i, m_i, max_rank - s)):
      1. [Jsk, Rsk] = qrcp_wide(M^sk(:, s:))                      (Alg. 1, Alg. 2)
      2. k = tri_rank(Rsk)                                       (Sec. 2.2)
      3. permute M(:, s:) (all m rows) and J(s:) by Jsk          (Sec. 3)
      4. k = 0: stop with rank s
      5. qr_tall = cholqr: M^pre = M(s:, s:s+k) Rsk(0:k,0:k)^{-1}; Cholesky
         QR; a breakdown at column t truncates k to t             (Alg. 3)
      6. Householder reconstruction -> Y, tau, D;
         R11 = diag(D) R^chol Rsk(0:k, 0:k)                      (Alg. 3, rows signed by D)
         (qr_tall = geqrf: Y, tau and R11 from GEQRF of M(s:, s:s+k))
      7. apply (I - Y T Y^T)^T to M(s:m, s+k:n)                  (Sec. 2.4, ORMQR)
      8. k < k_max or s + k_max = min(m, n, max_rank): stop with rank s + k
      9. M^sk(:, c:) = [Rsk12 - Rsk11 R11^{-1} R12; Rsk22]        (Alg. 1, Sec. 3)

    Any aspect ratio (Sec. 1.3): for m < n the loop ends after the block that
    reaches row m, and R is m x n upper trapezoidal.  ``max_rank`` (truncated
    output): the loop stops once max_rank columns are factored; the last block
    factors only the columns up to max_rank, and A(l:, l:) keeps the residual.
    """
    a = np.array(a, dtype=np.float64, order="F", copy=True)
    m, n = a.shape
    if qr_tall not in ("cholqr", "geqrf"):
        raise ValueError(qr_tall)
    lim = min(m, n) if max_rank is None else min(m, n, max(int(max_rank), 0))
    d = int(math.ceil(gamma * b - 1e-12))
    if msk is None:
        msk = sketch(a, d, seed, sketch_precision)
    else:
        msk = np.array(msk, dtype=np.float64, copy=True)
    jpiv = np.arange(n, dtype=np.int64)
    tau = np.zeros(min(m, n))
    ref = math.sqrt(float(np.max(np.sum(msk * msk, axis=0)))) if n else 0.0
    res = Result(a=a, jpiv=jpiv, tau=tau, rank=0)
    s = 0
    while s < lim:
        ni, mi = n - s, m - s
        kmax = min(b, ni, mi, lim - s)
        c = s + kmax
        cur = msk[:, s:]
        if not np.all(np.isfinite(cur)):
            res.status = ERR_NONFINITE
            res.rank = s
            return res
        if qrcp_wide == "lu":
            jsk, rsk, ipiv, margins = qrcp_wide_lu(cur, min(d, ni, mi))
        else:
            jsk, rsk, ipiv, margins = qrcp_wide_geqp3(cur, min(d, ni, mi))
        k = tri_rank(rsk, kmax, tol, ref)
        a[:, s:] = a[:, s + jsk]
        jpiv[s:] = jpiv[s + jsk]
        tr = BlockTrace(s=s, k=k, kmax=kmax, ipiv=ipiv, margins=margins, jsk=jsk,
                        msk_in=np.array(cur) if trace_sketch else None)
        res.trace.append(tr)
        if k == 0:
            res.rank = s
            return res
        if qr_tall == "geqrf":
            # ---- panel: Householder QR (GEQRF) of M(s:m, s:s+k) (Sec. 2.3) ----
            rp, y, tk = householder_qr(a[s:, s:s + k])
            blk = a[s:, s:s + k]
            blk[:, :] = np.tril(y, -1)
            blk[:k, :k] += np.triu(rp[:k, :k])
            tau[s:s + k] = tk
        else:
            # ---- panel: preconditioned Cholesky QR (Alg. 3) ----
            while True:
                mpre = solve_triangular(rsk[:k, :k], a[s:, s:s + k].T, trans="T", lower=False).T
                q, rc, keff = cholqr(mpre, cholqr_passes)
                if keff == k:
                    break
                k = keff              # breakdown: redo with the leading keff columns
                if k == 0:
                    tr.k = 0
                    res.rank = s
                    return res
            y, tk, dsig, _ = householder_reconstruct(q)
            r11 = dsig[:, None] * (rc @ rsk[:k, :k])
            # write Y below the diagonal and R11 on/above it
            blk = a[s:, s:s + k]
            blk[:, :] = y
            blk[:k, :k] = np.triu(r11) + np.tril(y[:k, :k], -1)
            tau[s:s + k] = tk
        tr.k = k
        # ---- trailing update M(s:m, s+k:n) <- Q^T M(s:m, s+k:n) ----
        if s + k < n:
            t = larft(y, tk)
            cmat = a[s:, s + k:]
            if trailing_precision == "f32":
                # the two products of the update run in FP32 (operands rounded
                # to FP32, FP32 accumulation); C itself stays FP64
                y32, t32, c32 = (x.astype(np.float32) for x in (y, t, cmat))
                w = t32.T @ (y32.T @ c32)
                a[s:, s + k:] = cmat - (y32 @ w).astype(np.float64)
            else:
                a[s:, s + k:] = apply_qt(y, t, cmat)
        if k < kmax or c >= lim:
            res.rank = s + k
            return res
        if max_blocks is not None and len(res.trace) >= max_blocks:
            # a leading sample of the loop (used to compare large problems
            # block-row by block-row); the trailing block is left updated
            res.rank = s + k
            return res
        # ---- sketch update (Alg. 1 last step; Sec. 3 "Sample update") ----
        rsk11 = rsk[:b, :b]
        r11b = np.triu(a[s:s + b, s:s + b])
        x = solve_triangular(r11b, rsk11.T, trans="T", lower=False).T   # Rsk11 R11^{-1}
        r12 = a[s:s + b, c:]
        rows = rsk.shape[0]
        new = np.zeros((d, n - c))
        new[:b] = rsk[:b, b:] - x @ r12
        new[b:rows] = np.triu(rsk[b:rows, b:])
        msk[:, c:] = new
        s = c
    res.rank = lim
    return res


# --------------------------------------------------------------------------
# Unpivoted Householder QR (the GEQRF baseline) and checking helpers.
# --------------------------------------------------------------------------
def geqrf(a: np.ndarray):
    """Unpivoted Householder QR in GEQRF storage: R on/above the diagonal,
    reflector vectors below, tau."""
    r, v, tau = householder_qr(a)
    out = np.array(r, order="F")
    kk = v.shape[1]
    for j in range(kk):
        out[j + 1:, j] = v[j + 1:, j]
    return out, tau


def form_q(af: np.ndarray, tau: np.ndarray, ncols: int | None = None) -> np.ndarray:
    """Explicit first ``ncols`` columns of Q = H_0 H_1 ... from GEQRF/GEQP3 storage."""
    m = af.shape[0]
    kk = len(tau)
    ncols = kk if ncols is None else ncols
    q = np.eye(m, ncols)
    for j in reversed(range(kk)):
        if tau[j] == 0.0:
            continue
        v = np.concatenate(([1.0], af[j + 1:, j]))
        q[j:, :] -= tau[j] * np.outer(v, v @ q[j:, :])
    return q


def upper_r(af: np.ndarray, rank: int) -> np.ndarray:
    """R (rank x n) read from GEQP3 storage."""
    return np.triu(af[:rank, :])


def residual_and_orth(a0: np.ndarray, res: Result):
    """||A P - Q_l R_l||_F / ||A||_F and ||Q_l^T Q_l - I||_F, with l = rank."""
    l = res.rank
    q = form_q(res.a, res.tau[:l], ncols=l) if l else np.zeros((a0.shape[0], 0))
    r = upper_r(res.a, l)
    ap = a0[:, res.jpiv]
    nrm = np.linalg.norm(a0)
    resid = np.linalg.norm(ap - q @ r) / (nrm if nrm else 1.0)
    orth = np.linalg.norm(q.T @ q - np.eye(l))
    return resid, orth


def canonical_flops(m: int, n: int) -> float:
    """GEQRF flop count used for the canonical rate (Sec. 1.4, LAWN 41):
    2 m n^2 - 2 n^3 / 3 for m >= n."""
    return 2.0 * m * n * n - 2.0 * n ** 3 / 3.0


def truncated_flops(m: int, n: int, l: int) -> float:
    """Householder QR of an m x n matrix stopped after l columns."""
    return 4.0 * m * n * l - 2.0 * (m + n) * l * l + (4.0 / 3.0) * l ** 3
