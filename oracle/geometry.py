"""Geometry of the simple interface problem on the bounding-box grid.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Follows the paper:
  * vertex-centred grid, nodes 0..N per axis, h = (hi - lo) / N     (Sec. 5.2)
  * node region: k if H_k(x) < 0, else 0 (exterior)               (Secs. 2.2, 5.1)
  * intersections of e_r-aligned grid segments with Gamma, found by
    bisection on H(x_1 + t (x_2 - x_1)) = 0                         (Sec. 5.1)
  * overlapping surface decomposition Gamma_r = {|n . e_r| > cos alpha};
    Gamma_r^h = intersections of Gamma_r with e_r-aligned lines      (Sec. 5.1)
  * reference plane Pi_i with i = argmax_j |n_j|                    (Sec. 5.1)
  * collocation points: PDE points on a degree-(p-2) lattice in d dims,
    Dirichlet points on a degree-p lattice and Neumann points on a
    degree-(p-1) lattice in the reference plane (d-1 dims)         (Sec. 5.4)
  * regular / irregular nodes of the FD stencil                      (Sec. 5.2)
  * closest-primary-point partition of unity                         (Sec. 5.3)
  * tensor-product Lagrange interpolation blocks                     (Sec. 5.5)

Where the paper leaves a choice open (the exact collocation lattice, the
stencil search window and its validity gate, the canonical order of the
surface points, tie rules, bisection length) the oracle takes the readings
written down in the design notes; the HIP library implements the same
readings independently.

Array conventions: a grid array has shape (N+1,)*d indexed [.., i1, i0]
(x fastest), so ``arr.ravel()`` is the linear node order
idx = i0 + (N+1) i1 (+ (N+1)^2 i2).
"""
import numpy as np
from scipy.spatial import cKDTree

from . import levelset

BISECT_STEPS = 52          # interval width 2^-52 of one grid segment
MARGIN = 3                 # outer node layers that must lie in region 0
TIE_BAND = 1e-12           # closest-centre tie band (relative, on squared distance)


class GeometryError(Exception):
    """Raised with .status in {'invalid', 'unresolved'}."""

    def __init__(self, status, msg):
        super().__init__(msg)
        self.status = status


# ----------------------------------------------------------------------------
# grid
# ----------------------------------------------------------------------------
def grid_h(prob):
    return (prob["hi"] - prob["lo"]) / prob["N"]


def node_coord_1d(prob):
    N = prob["N"]
    return prob["lo"] + np.arange(N + 1, dtype=np.float64) * grid_h(prob)


def mesh(prob):
    """Coordinates (x, y[, z]) of every node, each of grid shape."""
    d = prob["dim"]
    x1 = node_coord_1d(prob)
    n1 = x1.size
    out = []
    for a in range(d):
        shape = [1] * d
        shape[d - 1 - a] = n1
        out.append(np.broadcast_to(x1.reshape(shape), (n1,) * d))
    return tuple(out)


def node_regions(prob):
    """Region id per node: k (1-based) if H_k < 0, else 0 (Sec. 5.2, H = 0 is
    exterior).  Overlapping interiors or interfaces inside the outer MARGIN
    layers raise GeometryError('invalid')."""
    X = mesh(prob)
    d = prob["dim"]
    N = prob["N"]
    reg = np.zeros((N + 1,) * d, dtype=np.int8)
    for k, iface in enumerate(prob["ifaces"], start=1):
        inside = levelset.H(iface, X) < 0.0
        if np.any(inside & (reg != 0)):
            raise GeometryError("invalid", "interface interiors overlap")
        reg[inside] = k
    m = MARGIN
    inner = reg[(slice(m, N + 1 - m),) * d]
    if np.count_nonzero(reg) != np.count_nonzero(inner):
        raise GeometryError("invalid", "interface too close to the box boundary")
    return reg


# ----------------------------------------------------------------------------
# surface points (Sec. 5.1)
# ----------------------------------------------------------------------------
def transverse_axes(d, r):
    return [a for a in range(d) if a != r]


def surface_points(prob, reg):
    """Surface point set Gamma^h: intersections of family-r grid segments
    with every interface that satisfy |n_r| > cos alpha (Sec. 5.1), in
    canonical order (family r, line id, segment s, interface k), each marked
    primary or not (see primary()).  Line id of family r = i_b1 + (N+1) i_b2 over the
    transverse axes b1 < b2."""
    d, N = prob["dim"], prob["N"]
    K = len(prob["ifaces"])
    h = grid_h(prob)
    lo = prob["lo"]
    x1 = node_coord_1d(prob)
    L = (N + 1) ** (d - 1)
    rows = []   # (key, r, lid, s, k, ina, transverse index tuple)
    for r in range(d):
        A = np.moveaxis(reg, d - 1 - r, d - 1)      # along-r axis last
        a_side = A[..., :-1]
        b_side = A[..., 1:]
        T = transverse_axes(d, r)
        for k in range(1, K + 1):
            cross = (a_side == k) != (b_side == k)
            idx = np.nonzero(cross)
            # idx: transverse indices in reversed axis order, then s
            s = idx[-1]
            trans = idx[:-1][::-1]            # trans[j] is index along T[j]
            lid = np.zeros_like(s)
            mul = 1
            for j in range(d - 1):
                lid = lid + trans[j] * mul
                mul *= (N + 1)
            ina = a_side[idx] == k
            key = ((r * L + lid) * N + s) * K + (k - 1)
            for e in range(s.size):
                rows.append((int(key[e]), r, int(lid[e]), int(s[e]), k, bool(ina[e]),
                             tuple(int(trans[j][e]) for j in range(d - 1))))
    rows.sort(key=lambda t: t[0])
    nc = len(rows)
    fam = np.array([t[1] for t in rows], dtype=np.int64)
    lid = np.array([t[2] for t in rows], dtype=np.int64)
    seg = np.array([t[3] for t in rows], dtype=np.int64)
    kk = np.array([t[4] for t in rows], dtype=np.int64)
    ina = np.array([t[5] for t in rows], dtype=bool)
    pos = np.zeros((nc, d))
    for e, t in enumerate(rows):
        r = t[1]
        for j, b in enumerate(transverse_axes(d, r)):
            pos[e, b] = x1[t[6][j]]
    # bisection on t in [0, 1] along the segment (Sec. 5.1)
    xr0 = lo + seg.astype(np.float64) * h
    tlo = np.zeros(nc)
    thi = np.ones(nc)
    for k in range(1, K + 1):
        sel = kk == k
        if not np.any(sel):
            continue
        iface = prob["ifaces"][k - 1]
        f_sel = fam[sel]
        base = pos[sel].copy()
        a_lo = tlo[sel]
        a_hi = thi[sel]
        a_in = ina[sel]
        a_x0 = xr0[sel]
        for _ in range(BISECT_STEPS):
            mid = 0.5 * (a_lo + a_hi)
            P = base.copy()
            P[np.arange(P.shape[0]), f_sel] = a_x0 + mid * h
            inside = levelset.H(iface, tuple(P[:, a] for a in range(d))) < 0.0
            same = inside == a_in
            a_lo = np.where(same, mid, a_lo)
            a_hi = np.where(same, a_hi, mid)
        tlo[sel] = a_lo
        thi[sel] = a_hi
    troot = 0.5 * (tlo + thi)
    pos[np.arange(nc), fam] = xr0 + troot * h
    nrm = np.zeros((nc, d))
    for k in range(1, K + 1):
        sel = kk == k
        if np.any(sel):
            n = levelset.normal(prob["ifaces"][k - 1], tuple(pos[sel][:, a] for a in range(d)))
            nrm[sel] = np.stack(n, axis=1)
    keep = np.abs(nrm[np.arange(nc), fam]) > prob["cos_alpha"]
    return {
        "pos": pos[keep], "nrm": nrm[keep], "fam": fam[keep], "lid": lid[keep],
        "seg": seg[keep], "iface": kk[keep], "prim": primary(nrm[keep], fam[keep]),
        "n_candidates": nc,
    }


def primary(nrm, fam):
    """A surface point on a family-r line is primary (a DOF and a centre)
    when r = argmax_j |n_j| (lowest j on ties): the reference-plane rule of
    Sec. 5.1.  Every surface location is then carried by exactly one
    family; the other points of the overlapping set serve as collocation
    points only."""
    a = np.abs(nrm)
    best = a[:, 0].copy()
    arg = np.zeros(a.shape[0], dtype=np.int64)
    for j in range(1, a.shape[1]):
        m = a[:, j] > best
        best = np.where(m, a[:, j], best)
        arg = np.where(m, j, arg)
    return arg == fam


# ----------------------------------------------------------------------------
# collocation lattices (Sec. 5.4 rules (a)-(c))
# ----------------------------------------------------------------------------
def window(L):
    """1D set of L consecutive integers centred at 0 (extra point on +)."""
    a = -((L - 1) // 2)
    return list(range(a, a + L))


def stack_offset(j):
    """0, +1, -1, +2, -2, ... ."""
    if j == 0:
        return 0
    return (j + 1) // 2 if j % 2 == 1 else -(j // 2)


def lattice(D, m):
    """Unisolvent set for polynomials of degree m in D dims built by stacking
    parallel lines (planes) at offsets 0, +1, -1, ... that hold sets of degree
    m, m-1, ..., 0 (Radon's recursion).  The last coordinate is the stacking
    direction.  Size = C(m + D, D)."""
    if m < 0:
        return []
    if D == 0:
        return [()]
    if D == 1:
        return [(o,) for o in window(m + 1)]
    pts = []
    for j in range(m + 1):
        b = stack_offset(j)
        for q in lattice(D - 1, m - j):
            pts.append(tuple(q) + (b,))
    return pts


def shift_list(d, offs):
    """Window shifts tried in order for one lattice; only shifts s with -s in
    the lattice are allowed, so that the shifted window still contains offset
    0 and the centre stays its own collocation point."""
    if d == 2:
        cand = [(0,), (1,), (-1,), (2,), (-2,), (3,), (-3,), (4,), (-4,)]
    else:
        cand = [(a, b) for a in range(-4, 5) for b in range(-4, 5)]
        cand.sort(key=lambda s: (abs(s[0]) + abs(s[1]), abs(s[1]), -s[0], -s[1]))
    member = set(offs)
    return [s for s in cand if tuple(-v for v in s) in member]


def degree(prob):
    return 4 if prob["order"] == 4 else 2


def line_table(prob, surf):
    """For every (family, line id) the list of surface-point indices on it,
    in canonical order."""
    table = {}
    for i, (r, l) in enumerate(zip(surf["fam"].tolist(), surf["lid"].tolist())):
        table.setdefault((r, l), []).append(i)
    return table


def line_id(prob, r, coords):
    """Line id of the family-r line through integer transverse coordinates
    coords[b] (b != r)."""
    d, N = prob["dim"], prob["N"]
    T = transverse_axes(d, r)
    lid = 0
    mul = 1
    for b in T:
        lid += coords[b] * mul
        mul *= (N + 1)
    return lid


def _nearest(table, pos, ifc, ok, r, lid, i_ref, x_ref):
    """Index of the surface point on line (r, lid) of the interface of point
    i_ref, admissible by ok[], nearest to x_ref along e_r (lowest index on
    ties), and its distance; (-1, 0) if none."""
    bj, bd = -1, 0.0
    for j in table.get((r, lid), []):
        if ifc[j] != ifc[i_ref] or not ok[j]:
            continue
        dd = abs(pos[j][r] - x_ref)
        if bj < 0 or dd < bd:
            bj, bd = j, dd
    return bj, bd


def _pick(prob, table, pos, ifc, i, rs, a0, offs, s, need_prim=None):
    """Surface points of one shifted window, or None if any is invalid (or,
    with need_prim given, not primary)."""
    d, N = prob["dim"], prob["N"]
    h = grid_h(prob)
    T = transverse_axes(d, rs)
    allok = [True] * len(pos)
    sel = []
    for o in offs:
        ln = [a0[j] + o[j] + s[j] for j in range(d - 1)]
        if any(v < 0 or v > N for v in ln):
            return None
        coords = {b: ln[j] for j, b in enumerate(T)}
        bj, bd = _nearest(table, pos, ifc, allok, rs, line_id(prob, rs, coords), i, pos[i][rs])
        l1 = sum(abs(o[j] + s[j]) for j in range(d - 1))
        if bj < 0 or not (bd <= 2.0 * h * (float(l1) + 1.0)):
            return None
        if need_prim is not None and not need_prim[bj]:
            return None
        sel.append(bj)
    return sel


def stencils(prob, surf):
    """Dirichlet / Neumann collocation points (indices into the surface-point
    table) and PDE collocation points of every centre (every primary point is
    a centre; centres are numbered in canonical order).

    Reference plane: the one transverse to the centre's own family r, which
    is argmax_j |n_j| at a primary point (Sec. 5.1).  The centre is its own
    Dirichlet and Neumann point (offset 0), so every unknown enters its own
    local problem.  Transverse anchor a0 = floor(t + 1/2), t = (p - lo)/h on
    each transverse axis.  The point on line a0 + o + s is the surface point
    (primary or not) of the same interface on that family-r line nearest to
    p along e_r (lowest index on ties); it is valid when
    |delta| <= 2 h (|o + s|_1 + 1).

    Window shifts (rule (b) of Sec. 5.4: the two boundary sets stay
    together around the centre):
      (1) both windows moved by the same s, the first s of the Neumann
          lattice's shift list (each has -s in both lattices) for which every
          point of both is valid; when the Neumann data is a density (every
          kind but the interior Dirichlet problem) a first pass over the list
          takes primary Neumann points only;
      (2) if no common shift exists, each lattice on its own: the first valid
          shift of its own list (the Neumann lattice again primary-only first
          when its data is a density).
    None -> GeometryError('unresolved')."""
    d = prob["dim"]
    p = degree(prob)
    h = grid_h(prob)
    lo = prob["lo"]
    offD = lattice(d - 1, p)
    offN = lattice(d - 1, p - 1)
    offP = lattice(d, p - 2)
    SD = shift_list(d, offD)
    SN = shift_list(d, offN)
    table = line_table(prob, surf)
    pos = surf["pos"].tolist()
    fam = surf["fam"].tolist()
    ifc = surf["iface"].tolist()
    primlist = surf["prim"].tolist()
    n_density = prob.get("bie", "interface") != "dirichlet"
    npasses = (primlist, None) if n_density else (None,)
    cen = np.nonzero(surf["prim"])[0]
    Nb = cen.size
    Didx = np.zeros((Nb, len(offD)), dtype=np.int64)
    Nidx = np.zeros((Nb, len(offN)), dtype=np.int64)
    shD = np.zeros(Nb, dtype=np.int64)
    shN = np.zeros(Nb, dtype=np.int64)
    for c, i in enumerate(cen.tolist()):
        rs = fam[i]
        T = transverse_axes(d, rs)
        a0 = [int(np.floor((pos[i][b] - lo) / h + 0.5)) for b in T]
        done = False
        # (1) one shift for both windows
        for req in npasses:
            for si, s in enumerate(SN):
                selD = _pick(prob, table, pos, ifc, i, rs, a0, offD, s, None)
                if selD is None:
                    continue
                selN = _pick(prob, table, pos, ifc, i, rs, a0, offN, s, req)
                if selN is None:
                    continue
                Didx[c], Nidx[c] = selD, selN
                shD[c] = shN[c] = si
                done = True
                break
            if done:
                break
        if done:
            continue
        # (2) each lattice on its own (shift numbers offset by 100)
        for out, sh, offs, SL, passes in ((Didx, shD, offD, SD, (None,)), (Nidx, shN, offN, SN, npasses)):
            found = False
            for req in passes:
                for si, s in enumerate(SL):
                    sel = _pick(prob, table, pos, ifc, i, rs, a0, offs, s, req)
                    if sel is not None:
                        out[c] = sel
                        sh[c] = 100 + si
                        found = True
                        break
                if found:
                    break
            if not found:
                raise GeometryError("unresolved", "no valid collocation stencil for centre %d" % c)
    P = surf["pos"][cen]
    pde = np.zeros((Nb, len(offP), d))
    for j, o in enumerate(offP):
        for a in range(d):
            pde[:, j, a] = P[:, a] + float(o[a]) * h
    return {"D": Didx, "N": Nidx, "shiftD": shD, "shiftN": shN,
            "pde_pts": pde, "offP": offP, "offD": offD, "offN": offN}


EXT_SHIFTS = (0, 1, -1, 2, -2)
EXT_OWN = (-1, 1, -2, 2, -3, 3, -4, 4)


def _lagrange(u, nodes):
    """Lagrange basis values at u for the given (float) nodes."""
    out = []
    for j, xj in enumerate(nodes):
        wj = 1.0
        for m, xm in enumerate(nodes):
            if m != j:
                wj = wj * (u - xm) / (xj - xm)
        out.append(wj)
    return out


def extension(prob, surf, st):
    """Values of the density at the non-primary surface points used as
    Neumann collocation points (and as Dirichlet points when a density is
    the jump [u]: interior Dirichlet problems and the two-density
    formulation), as combinations of primary values by degree
    p-1 Lagrange interpolation along one grid direction on the surface.

    Candidate stencils for a non-primary point q on a family-r line (its
    coordinates off axis r are grid values), in this order:
      (i)  for s in (0, 1, -1, 2, -2): the p lines of family
           r' = argmax_j |n_j(q)| at integer e_r positions base+s ..
           base+s+p-1, base = floor(t) - (p/2 - 1), t = (x_r - lo)/h, through
           q's other grid coordinates; nodes = those positions, evaluated at t;
      (ii) for each transverse axis b of r (increasing): the family-r lines
           through q's line moved by o e_b, o taken from (-1, 1, -2, 2, -3, 3,
           -4, 4) in that order, the first p offsets whose line carries a
           valid point; nodes = the offsets, evaluated at 0.
    On each line the primary point of the same interface nearest to q along
    e_F (F the family of the lines) is taken, valid when
    |delta| <= 2 h (|o| + 1), o the line's offset from floor(t) (i) or from
    q's line (ii).  Among the fully valid candidates the one with the
    smallest sum_j |w_j| (summed in node order) is used, the first in the
    order above on ties; none -> GeometryError('unresolved').

    Returns (idx, w) of shape (n_surf, p): psi_S[q] = sum_j w[q,j] psi[idx[q,j]]
    (idx = -1, w = 0 where unused; a primary point maps to itself)."""
    d, N = prob["dim"], prob["N"]
    p = degree(prob)
    h = grid_h(prob)
    lo = prob["lo"]
    ns = surf["pos"].shape[0]
    prim = surf["prim"]
    dof_of = np.cumsum(prim) - 1
    idx = np.full((ns, p), -1, dtype=np.int64)
    w = np.zeros((ns, p))
    idx[prim, 0] = dof_of[prim]
    w[prim, 0] = 1.0
    need = np.zeros(ns, dtype=bool)
    need[st["N"].ravel()] = True
    if prob.get("bie") in ("dirichlet", "two_density"):
        # a density is the jump [u]: it enters at the Dirichlet points
        need[st["D"].ravel()] = True
    need &= ~prim
    table = line_table(prob, surf)
    pos = surf["pos"].tolist()
    ifc = surf["iface"].tolist()
    okp = prim.tolist()

    def point_on(q, F, coords, axis, o, oref):
        c = dict(coords)
        c[axis] = c[axis] + o
        if c[axis] < 0 or c[axis] > N:
            return -1
        bj, bd = _nearest(table, pos, ifc, okp, F, line_id(prob, F, c), q, pos[q][F])
        if bj < 0 or not (bd <= 2.0 * h * (float(abs(o - oref)) + 1.0)):
            return -1
        return bj

    for q in np.nonzero(need)[0].tolist():
        r = int(surf["fam"][q])
        n = surf["nrm"][q]
        rp = 0
        best = abs(n[0])
        for a in range(1, d):
            if abs(n[a]) > best:
                best = abs(n[a])
                rp = a
        grid = {b: int(np.floor((pos[q][b] - lo) / h + 0.5)) for b in range(d) if b != r}
        t = (pos[q][r] - lo) / h
        ft = int(np.floor(t))
        base = ft - (p // 2 - 1)
        cands = []
        for s in EXT_SHIFTS:
            c = dict(grid)
            c[r] = 0
            offs = [base + s + j for j in range(p)]
            sel = [point_on(q, rp, c, r, o, ft) for o in offs]
            if min(sel) >= 0:
                cands.append((sel, _lagrange(t, [float(o) for o in offs])))
        for b in transverse_axes(d, r):
            sel, offs = [], []
            for o in EXT_OWN:
                j = point_on(q, r, grid, b, o, 0)
                if j >= 0:
                    sel.append(j)
                    offs.append(o)
                    if len(sel) == p:
                        break
            if len(sel) == p:
                cands.append((sel, _lagrange(0.0, [float(o) for o in offs])))
        if not cands:
            raise GeometryError("unresolved", "no interpolation stencil for surface point %d" % q)
        bestc, bestL = None, 0.0
        for sel, wts in cands:
            L = 0.0
            for x in wts:
                L = L + abs(x)
            if bestc is None or L < bestL:
                bestc, bestL = (sel, wts), L
        sel, wts = bestc
        for j in range(p):
            idx[q, j] = dof_of[sel[j]]
            w[q, j] = wts[j]
    return idx, w


# ----------------------------------------------------------------------------
# FD stencil support, irregular nodes (Sec. 5.2)
# ----------------------------------------------------------------------------
def stencil_offsets(prob):
    """Offsets of the FD stencil: 5/7-point for order 2, 9/27-point for order 4."""
    d = prob["dim"]
    offs = []
    for o in np.ndindex(*(3,) * d):
        o = tuple(v - 1 for v in o[::-1])    # o[0] is the x offset
        if all(v == 0 for v in o):
            continue
        if prob["order"] == 2 and sum(abs(v) for v in o) != 1:
            continue
        offs.append(o)
    return offs


def _shift(arr, o, d):
    """arr shifted so that out[P] = arr[P + o] on interior nodes (edges cut)."""
    sl = []
    for a in range(d - 1, -1, -1):
        sl.append(slice(1 + o[a], arr.shape[d - 1 - a] - 1 + o[a]))
    return arr[tuple(sl)]


def irregular_nodes(prob, reg):
    """Linear indices of interior nodes whose stencil contains a node of
    another region (the set I_h of Sec. 5.2), increasing."""
    d, N = prob["dim"], prob["N"]
    core = reg[(slice(1, N),) * d]
    irr = np.zeros(core.shape, dtype=bool)
    for o in stencil_offsets(prob):
        irr |= _shift(reg, o, d) != core
    full = np.zeros(reg.shape, dtype=bool)
    full[(slice(1, N),) * d] = irr
    return np.nonzero(full.ravel())[0]


def unravel(idx, prob):
    """Linear node index -> index tuple (i0, i1[, i2])."""
    n1 = prob["N"] + 1
    out = []
    for _ in range(prob["dim"]):
        out.append(idx % n1)
        idx = idx // n1
    return out


def ravel(ind, prob):
    n1 = prob["N"] + 1
    idx = np.zeros_like(ind[0])
    mul = 1
    for a in range(prob["dim"]):
        idx = idx + ind[a] * mul
        mul *= n1
    return idx


def interp_blocks(prob, dofs):
    """Start index per axis of the (q+1)^d interpolation block of every DOF:
    q + 1 consecutive nodes centred at floor(t + 1/2), clamped to [0, N - q]
    (Sec. 5.5); q = p."""
    q = degree(prob)
    N = prob["N"]
    h = grid_h(prob)
    t = (dofs["pos"] - prob["lo"]) / h
    st = np.floor(t + 0.5).astype(np.int64) - q // 2
    return np.clip(st, 0, N - q)


def correction_entries(prob, reg, irr, dofs, blocks):
    """(interface k, node) pairs at which the partition-of-unity value
    C^(k) is needed, ordered k-major, node-minor.  Needed by the RHS
    correction (Sec. 5.2 and the multi-crossing remark: C = C^(reg P) -
    C^(reg Q), C^(0) = 0) and, in the corrected interpolation (Sec. 5.5), at
    the block nodes of a DOF on interface k that lie inside another interface
    k' (the DOF's own side is corrected with its own local polynomial, so
    only C^(k') is needed there)."""
    d, N = prob["dim"], prob["N"]
    K = len(prob["ifaces"])
    flat = reg.ravel()
    need = np.zeros((K + 1, flat.size), dtype=bool)
    ind = unravel(irr, prob)
    rp = flat[irr]
    for o in stencil_offsets(prob):
        q = ravel([ind[a] + o[a] for a in range(d)], prob)
        rq = flat[q]
        m = rq != rp
        need[rp[m], q[m]] = True
        need[rq[m], q[m]] = True
    q1 = degree(prob) + 1
    for blk in np.ndindex(*(q1,) * d):
        ind_b = [blocks[:, a] + blk[a] for a in range(d)]
        q = ravel(ind_b, prob)
        rq = flat[q]
        k = dofs["iface"]
        m = (rq != k) & (rq != 0)
        need[rq[m], q[m]] = True
    need[0] = False
    kk, nodes = np.nonzero(need)
    return kk.astype(np.int64), nodes.astype(np.int64)


def closest_centres(prob, dofs, kk, nodes):
    """Owner centre of every correction entry: among the centres of interface
    k, the one nearest to the node (squared distance dx*dx + dy*dy (+dz*dz));
    among those within d2 <= d2min (1 + 1e-12) the lowest canonical index
    (Sec. 5.3, closest-point weight)."""
    d = prob["dim"]
    h = grid_h(prob)
    lo = prob["lo"]
    ind = unravel(nodes, prob)
    X = np.stack([lo + ind[a].astype(np.float64) * h for a in range(d)], axis=1)
    owner = np.full(nodes.size, -1, dtype=np.int64)
    P = dofs["pos"]
    for k in np.unique(kk):
        cid = np.nonzero(dofs["iface"] == k)[0]
        if cid.size == 0:
            raise GeometryError("unresolved", "interface %d has no surface points" % k)
        tree = cKDTree(P[cid])
        sel = np.nonzero(kk == k)[0]
        dist, _ = tree.query(X[sel], k=1)
        for e, rad in zip(sel.tolist(), dist.tolist()):
            cand = cid[tree.query_ball_point(X[e], rad * (1.0 + 1e-9) + 1e-300)]
            dx = X[e][None, :] - P[cand]
            d2 = dx[:, 0] * dx[:, 0] + dx[:, 1] * dx[:, 1]
            if d == 3:
                d2 = d2 + dx[:, 2] * dx[:, 2]
            m = d2.min()
            ok = d2 <= m * (1.0 + TIE_BAND)
            owner[e] = cand[ok].min()
    return owner


def closest_centres_brute(prob, dofs, kk, nodes):
    """Brute-force version of closest_centres (used only as a pin)."""
    d = prob["dim"]
    h = grid_h(prob)
    lo = prob["lo"]
    ind = unravel(nodes, prob)
    owner = np.full(nodes.size, -1, dtype=np.int64)
    P = dofs["pos"]
    for e in range(nodes.size):
        cid = np.nonzero(dofs["iface"] == kk[e])[0]
        x = [lo + float(ind[a][e]) * h for a in range(d)]
        d2 = (x[0] - P[cid, 0]) * (x[0] - P[cid, 0]) + (x[1] - P[cid, 1]) * (x[1] - P[cid, 1])
        if d == 3:
            d2 = d2 + (x[2] - P[cid, 2]) * (x[2] - P[cid, 2])
        m = d2.min()
        owner[e] = cid[d2 <= m * (1.0 + TIE_BAND)].min()
    return owner


def build(prob):
    """Full geometry set-up (step S0): regions, surface points, centres
    (primary points), stencils, density extension, irregular nodes,
    interpolation blocks, correction entries and their owners."""
    if prob["N"] & (prob["N"] - 1) or prob["N"] < 8:
        raise GeometryError("invalid", "N must be a power of two >= 8")
    reg = node_regions(prob)
    surf = surface_points(prob, reg)
    cen = np.nonzero(surf["prim"])[0]
    if cen.size == 0:
        raise GeometryError("invalid", "no surface points")
    dofs = {"sidx": cen, "pos": surf["pos"][cen], "nrm": surf["nrm"][cen],
            "fam": surf["fam"][cen], "iface": surf["iface"][cen]}
    st = stencils(prob, surf)
    ext_idx, ext_w = extension(prob, surf, st)
    irr = irregular_nodes(prob, reg)
    blocks = interp_blocks(prob, dofs)
    kk, nodes = correction_entries(prob, reg, irr, dofs, blocks)
    owner = closest_centres(prob, dofs, kk, nodes)
    return {"prob": prob, "h": grid_h(prob), "reg": reg, "surf": surf, "dofs": dofs, "st": st,
            "ext_idx": ext_idx, "ext_w": ext_w,
            "irr": irr, "blocks": blocks, "ck": kk, "cnode": nodes, "cowner": owner}
