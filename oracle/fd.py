"""Finite-difference operators and the box solver (paper Sec. 5.2).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Operators (h-scaled, kappa = reduced reaction coefficient):
  order 4, 2D  A_h = D_x + D_y + h^2/6 D_x D_y - kappa (I + h^2/12 Lap_5)
               (eq. 9p-cds written in tensor form), RHS B_h f = f + h^2/12 Lap_5 f
  order 4, 3D  A_h = sum D_k + h^2/6 sum_{j<k} D_j D_k + h^4/48 D_x D_y D_z
                     - kappa (I + h^2/12 Lap_7)   (eq. 27p-cds), B_h = I + h^2/12 Lap_7
  order 2      A_h = Lap_5 / Lap_7 - kappa I, B_h = I   (2nd-order variant)
with D_k the 3-point second difference along axis k.  A test checks the
tensor form against the coefficients printed in eqs. 9p-cds and 27p-cds.

The box solve (Alg. 1 Step 3.3: "with FFT") diagonalises A_h with homogeneous
Dirichlet data by the type-I discrete sine transform on the interior nodes.
"""
import itertools

import numpy as np
import scipy.fft
import scipy.sparse
import scipy.sparse.linalg


def _tensor(parts):
    """Tensor product of 1D stencils {offset: coef}: parts[a] acts on axis a."""
    out = {}
    for combo in itertools.product(*[list(p.items()) for p in parts]):
        off = tuple(c[0] for c in combo)
        val = 1.0
        for c in combo:
            val *= c[1]
        out[off] = out.get(off, 0.0) + val
    return out


def _add(st, other, w):
    for k, v in other.items():
        st[k] = st.get(k, 0.0) + w * v


def stencils(d, order, h, kappa):
    """(A_h, B_h) as dicts {offset (ox, oy[, oz]): coefficient}."""
    D = {-1: 1.0 / (h * h), 0: -2.0 / (h * h), 1: 1.0 / (h * h)}
    I = {0: 1.0}
    Dk = []
    for a in range(d):
        Dk.append(_tensor([D if b == a else I for b in range(d)]))
    lap = {}
    for a in range(d):
        _add(lap, Dk[a], 1.0)
    ident = _tensor([I] * d)
    if order == 2:
        A = dict(lap)
        _add(A, ident, -kappa)
        return A, ident
    L = dict(lap)
    for a in range(d):
        for b in range(a + 1, d):
            _add(L, _tensor([D if c in (a, b) else I for c in range(d)]), h * h / 6.0)
    if d == 3:
        _add(L, _tensor([D, D, D]), h ** 4 / 48.0)
    B = dict(ident)
    _add(B, lap, h * h / 12.0)
    A = dict(L)
    _add(A, B, -kappa)
    A = {k: v for k, v in A.items() if v != 0.0}
    B = {k: v for k, v in B.items() if v != 0.0}
    return A, B


def _view(arr, o, d):
    """Interior view of arr shifted by offset o (o[0] along x)."""
    sl = []
    for j in range(d):
        a = d - 1 - j
        sl.append(slice(1 + o[a], arr.shape[j] - 1 + o[a]))
    return arr[tuple(sl)]


def apply(st, v):
    """Interior values of sum_o c_o v(P + o) for a full grid array v."""
    d = v.ndim
    out = np.zeros(tuple(s - 2 for s in v.shape))
    for o, c in st.items():
        out += c * _view(v, o, d)
    return out


def eigenvalues(d, order, N, h, kappa):
    """Eigenvalues of A_h on sin modes k = 1..N-1 per axis, as a grid
    (indexed [.., k1, k0])."""
    k = np.arange(1, N)
    s1 = -4.0 / (h * h) * np.sin(k * np.pi / (2 * N)) ** 2
    S = []
    for a in range(d):
        shape = [1] * d
        shape[d - 1 - a] = N - 1
        S.append(s1.reshape(shape))
    lap = sum(S)
    if order == 2:
        return lap - kappa + np.zeros((N - 1,) * d)
    pair = 0.0
    for a in range(d):
        for b in range(a + 1, d):
            pair = pair + S[a] * S[b]
    lam = lap + h * h / 6.0 * pair
    if d == 3:
        lam = lam + h ** 4 / 48.0 * S[0] * S[1] * S[2]
    return lam - kappa * (1.0 + h * h / 12.0 * lap) + np.zeros((N - 1,) * d)


def dst_solve(F, d, order, N, h, kappa):
    """Solve A_h v = F on the interior nodes with v = 0 on the box boundary
    (exact, by the type-I DST)."""
    lam = eigenvalues(d, order, N, h, kappa)
    Fh = scipy.fft.dstn(F, type=1)
    return scipy.fft.idstn(Fh / lam, type=1)


def sparse_matrix(d, order, N, h, kappa):
    """A_h on the (N-1)^d interior unknowns as a sparse matrix (pin only)."""
    A, _ = stencils(d, order, h, kappa)
    n1 = N - 1
    n = n1 ** d
    idx = np.arange(n).reshape((n1,) * d)
    rows, cols, vals = [], [], []
    for o, c in A.items():
        src = [slice(None)] * d
        dst = [slice(None)] * d
        for j in range(d):
            a = d - 1 - j
            if o[a] > 0:
                src[j] = slice(0, n1 - o[a]); dst[j] = slice(o[a], n1)
            elif o[a] < 0:
                src[j] = slice(-o[a], n1); dst[j] = slice(0, n1 + o[a])
        r = idx[tuple(src)].ravel()
        cc = idx[tuple(dst)].ravel()
        rows.append(r); cols.append(cc); vals.append(np.full(r.size, c))
    return scipy.sparse.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                                   shape=(n, n))


def lu_solve(F, d, order, N, h, kappa):
    """Sparse-LU solve of the same system (pin only)."""
    A = sparse_matrix(d, order, N, h, kappa)
    return scipy.sparse.linalg.spsolve(A.tocsc(), F.ravel()).reshape(F.shape)
