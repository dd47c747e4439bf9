"""Plain NumPy transcription of the ANKH-FMM evaluation (test infrastructure only).

Follows the paper's steps in its order and notation, with no blocking or
fusion: tree (perfect octree of depth E), modified charges Q_s by Alg. 2
(Chebyshev basis S = H T, derivatives S^(n) = H D^n T), upward M2M, far field
by M2L over the interaction lists of every level including the cells of the
adjacent periodic images, far periodic images through one root operator,
near field by direct pair sums over adjacent leaves, self energy and the
neutralising background.  Forces and fields follow from the adjoint
(L2L = M2M^T, L2P = P2M^T, gradients of the pair terms).

Readings of the paper taken here (each also listed in the design notes):
* Chebyshev nodes r_k = cos((2k+1) pi / (2L)), k = 0..L-1 (the printed node
  formula lacks pi and mixes index bases).
* The differentiation matrix D with T' = D T is strictly lower triangular:
  T'_n = 2n sum_{j<n, n-j odd} T_j / c_j, c_0 = 2, c_j = 1 otherwise.
* S^(n)(y) = (2/w)^n H D^n T(y_hat), y_hat = (y - ctr)/(w/2); the loop of
  Alg. 2 takes S^(0) = H T before the first application of D.
* Theta enters D_y = q + mu.grad + Theta:grad grad literally; off-diagonal
  terms therefore appear twice (as Alg. 2 does).
* The root (far image) operator C_per = sum over images I in Z_p with
  |I|_inf >= 2 of the root-to-image M2L matrix, built directly on the root's
  Chebyshev grid (the equispaced grid and FFT of the periodicity section only
  accelerate the same sum).
* E_rec is dropped (small xi); the background -pi Q^2/(2 V xi^2) is added for
  non-neutral cells.

ANKH-FFT (far="fft"): the leaf modified charges are reinterpolated onto an
equispaced grid per leaf (Le nodes per axis spanning the leaf), and the far
energy 1/2 v^T A v over all non-adjacent leaf pairs is evaluated in the
Fourier domain, 1/2 (1/N) sum D |F6 chi v|^2 with D = F6 applied to the
generating entries of A.  Readings taken here:
* the grid spans the leaf (the node spacing of the diagonal-construction
  algorithm; the printed grid radius is half of that);
* the leaf grid is periodic, so the cell dimensions of the 6D transform are
  circular of length 2^E with no padding; the node dimensions are padded to
  2 Le - 1 (node differences -(Le-1)..Le-1);
* the image sum of each entry runs over the source-cell displacements
  within n (p + 1/2) cells per axis, which keeps each entry a function of
  the cell difference modulo n; adjacent displacements (the near field) are
  excluded, and the far images need no separate root operator.

The near-field pair sums use the pinned pair routine of `ewald.c`
(`oracle_near_field`).  Parameters (depth E, order L, xi, image radius p) are
inputs: this module chooses nothing.
"""
from __future__ import annotations

import ctypes
import itertools
import math

import numpy as np
from scipy.special import erfc

from . import lib as _oracle_lib, _p, _c64


# ---- 1D Chebyshev tools (ANKH-FMM numerical differentiation section) --------

def cheb_nodes(L: int) -> np.ndarray:
    k = np.arange(L)
    return np.cos((2 * k + 1) * np.pi / (2 * L))


def cheb_T(x, L: int) -> np.ndarray:
    """T_0..T_{L-1} at x by the three-term recurrence; shape x.shape + (L,)."""
    x = np.asarray(x, dtype=np.float64)
    T = np.empty(x.shape + (L,))
    T[..., 0] = 1.0
    if L > 1:
        T[..., 1] = x
    for m in range(2, L):
        T[..., m] = 2 * x * T[..., m - 1] - T[..., m - 2]
    return T


def cheb_H(L: int) -> np.ndarray:
    """H[k, m] = (1/L) (1 if m = 0 else 2 T_m(r_k)), so that S(x) = H T(x)."""
    Tr = cheb_T(cheb_nodes(L), L)
    H = 2.0 * Tr / L
    H[:, 0] = 1.0 / L
    return H


def cheb_D(L: int) -> np.ndarray:
    """T'(x) = D T(x)."""
    D = np.zeros((L, L))
    for n in range(1, L):
        for j in range(n):
            if (n - j) % 2 == 1:
                D[n, j] = 2.0 * n / (2.0 if j == 0 else 1.0)
    return D


def lagrange_derivs(xhat, L: int, nmax: int, h: float) -> np.ndarray:
    """S^(n)_k at scaled coordinates xhat for n = 0..nmax, with physical
    scaling (1/h)^n; shape xhat.shape + (nmax+1, L)."""
    H, D = cheb_H(L), cheb_D(L)
    T = cheb_T(xhat, L)
    out = np.empty(np.shape(xhat) + (nmax + 1, L))
    Tn = T
    for n in range(nmax + 1):
        out[..., n, :] = (Tn @ H.T) / h ** n
        Tn = Tn @ D.T
    return out


# ---- kernel ------------------------------------------------------------------

def kernel_H(r, xi: float) -> np.ndarray:
    r = np.asarray(r, dtype=np.float64)
    return erfc(xi * r) / r


# ---- tree --------------------------------------------------------------------

def wrap(pos, edge):
    r = 0.5 * edge
    out = pos - edge * np.floor((pos + r) / edge)
    out[out >= r] -= edge
    return out


def leaf_index(pos_wrapped, edge, depth, nside=None):
    """Leaf (i, j, k) of each wrapped position; nside leaves per axis (default 2^depth)."""
    n = (1 << depth) if nside is None else int(nside)
    w = edge / n
    ijk = np.floor((pos_wrapped + 0.5 * edge) / w).astype(np.int64)
    return np.clip(ijk, 0, n - 1)


# ---- operators ---------------------------------------------------------------

def nodes3d(L: int) -> np.ndarray:
    r = cheb_nodes(L)
    g = np.stack(np.meshgrid(r, r, r, indexing="ij"), axis=-1)
    return g.reshape(-1, 3)


def m2m_1d(Lp: int, Lc: int | None = None):
    """V[b][a, i] = S_a(child node i in parent coordinates), b = 0 low, 1 high child;
    parent order Lp, child order Lc (equal on the octree levels; the root may be finer)."""
    Lc = Lp if Lc is None else Lc
    r = cheb_nodes(Lc)
    H = cheb_H(Lp)
    lo = cheb_T((r - 1) / 2, Lp) @ H.T     # [i, a]
    hi = cheb_T((r + 1) / 2, Lp) @ H.T
    return [lo.T.copy(), hi.T.copy()]


def interaction_offsets():
    return [d for d in itertools.product(range(-3, 4), repeat=3) if max(abs(c) for c in d) >= 2]


def m2l_matrix(d, w: float, L: int, xi: float) -> np.ndarray:
    """C[t, s]_{kl} = H(x_k^t, y_l^s) for the source cell at offset d (cells of width w)."""
    g = nodes3d(L)
    diff = 0.5 * w * (g[:, None, :] - g[None, :, :]) - w * np.asarray(d, dtype=np.float64)
    return kernel_H(np.sqrt(np.sum(diff * diff, axis=-1)), xi)


def periodic_root_matrix(edge: float, L: int, xi: float, p: int) -> np.ndarray:
    """sum over images I in Z_p with |I|_inf >= 2 of H(x_k - x_l - edge I) on the root grid."""
    g = nodes3d(L) * (0.5 * edge)
    base = g[:, None, :] - g[None, :, :]
    C = np.zeros((len(g), len(g)))
    for I in itertools.product(range(-p, p + 1), repeat=3):
        if max(abs(c) for c in I) < 2:
            continue
        diff = base - edge * np.asarray(I, dtype=np.float64)
        C += kernel_H(np.sqrt(np.sum(diff * diff, axis=-1)), xi)
    return C


def _valid_mask(n, d):
    idx = np.arange(n)
    masks = []
    for c in d:
        even = idx % 2 == 0
        m = np.ones(n, dtype=bool)
        if c == 3:
            m = even
        elif c == -3:
            m = ~even
        masks.append(m)
    return masks[0][:, None, None] & masks[1][None, :, None] & masks[2][None, None, :]


# ---- ANKH-FFT far field (the ANKH-FFT section) -------------------------------

def equi_nodes(Le: int) -> np.ndarray:
    """Equispaced nodes of a leaf in scaled coordinates: -1 + 2a/(Le - 1), a = 0..Le-1.  The grid
    spans the whole leaf (the node spacing of the diagonal-construction algorithm, 2v/(L-1) with v
    the leaf half-width), so adjacent leaves share their face nodes."""
    return -1.0 + 2.0 * np.arange(Le) / (Le - 1)


def equi_lagrange(x, Le: int) -> np.ndarray:
    """U_a(x), the Lagrange polynomials of the equispaced nodes; shape x.shape + (Le,)."""
    t = equi_nodes(Le)
    x = np.asarray(x, dtype=np.float64)
    out = np.ones(x.shape + (Le,))
    for a in range(Le):
        for b in range(Le):
            if b != a:
                out[..., a] *= (x - t[b]) / (t[a] - t[b])
    return out


def equi_reinterp(L: int, Le: int) -> np.ndarray:
    """E[a, k] = U_a(r_k): maps the modified charges of the Chebyshev nodes r_k of a leaf to those
    of its equispaced nodes (H(r_k, .) ~ sum_a U_a(r_k) H(x_a, .))."""
    return equi_lagrange(cheb_nodes(L), Le).T.copy()


def fft_node_period(Le: int) -> int:
    """Length of the node dimensions of the transform: node differences span -(Le-1)..Le-1."""
    return 2 * Le - 1


def fft_kernel_table(n: int, w: float, Le: int, xi: float, p: int) -> np.ndarray:
    """The generating entries of the far-field matrix A in circulant order, K[gx, ax, gy, ay, gz, az]:
    cell residue g (mod n = 2^E) and node difference a (mod Pa = 2Le - 1) per axis.  The entry sums
    H over the images of the source cell whose cell displacement D = g - n I has |D_axis| <= n (p + 1/2)
    on every axis and is not adjacent (max |D| >= 2, the leaf pairs the direct near field does not
    take); the displacement of the two nodes is D w + a h, h = w / (Le - 1)."""
    Pa = fft_node_period(Le)
    h = w / (Le - 1)
    da = np.arange(-(Le - 1), Le)
    lim = n * (p + 0.5)
    disp = {g: [g - n * I for I in range(-p - 2, p + 3) if abs(g - n * I) <= lim] for g in range(n)}
    K = np.zeros((n, Pa, n, Pa, n, Pa))
    idx = da % Pa
    for gx, gy, gz in itertools.product(range(n), repeat=3):
        acc = np.zeros((len(da),) * 3)
        for Dx in disp[gx]:
            for Dy in disp[gy]:
                for Dz in disp[gz]:
                    if max(abs(Dx), abs(Dy), abs(Dz)) < 2:
                        continue
                    zx, zy, zz = Dx * w + da * h, Dy * w + da * h, Dz * w + da * h
                    r = np.sqrt(zx[:, None, None] ** 2 + zy[None, :, None] ** 2 + zz[None, None, :] ** 2)
                    acc += kernel_H(r, xi)
        K[gx, :, gy, :, gz, :][np.ix_(idx, idx, idx)] = acc
    return K


def fft_far(Q, n: int, L: int, Le: int, K) -> tuple:
    """ANKH-FFT far field from the leaf modified charges Q [n^3, L^3] (leaves in lexicographic order):
    M = E Q on the equispaced grids, v = the zero-padded 6D array chi v, w = F6 v, D = F6 K (real),
    energy 1/2 (1/N) sum D |w|^2 and the leaf local expansions Lambda = E^T chi^T F6^-1 (D w)."""
    Pa = fft_node_period(Le)
    E = equi_reinterp(L, Le)
    M = np.einsum("ai,bj,ck,xyzijk->xyzabc", E, E, E, Q.reshape(n, n, n, L, L, L))
    X = np.zeros((n, Pa, n, Pa, n, Pa))
    X[:, :Le, :, :Le, :, :Le] = M.transpose(0, 3, 1, 4, 2, 5)
    D = np.fft.fftn(K)
    W = np.fft.fftn(X)
    energy = 0.5 * float(np.sum(D.real * np.abs(W) ** 2)) / X.size
    phi = np.fft.ifftn(D * W).real[:, :Le, :, :Le, :, :Le].transpose(0, 2, 4, 1, 3, 5)
    Lam = np.einsum("ai,bj,ck,xyzabc->xyzijk", E, E, E, phi)
    return energy, Lam.reshape(n ** 3, L ** 3), D


def fft_far_dense(Q, n: int, w: float, L: int, Le: int, xi: float, p: int) -> float:
    """The same far energy by its definition (tiny cases): 1/2 sum over leaf pairs (t, s) and the
    images of s within the displacement cube, not adjacent to t, of M_t^T G M_s, G[a, b] = H between
    the equispaced nodes."""
    E = equi_reinterp(L, Le)
    M = np.einsum("ai,bj,ck,xyzijk->xyzabc", E, E, E, Q.reshape(n, n, n, L, L, L)).reshape(n ** 3, Le ** 3)
    g = np.stack(np.meshgrid(*(equi_nodes(Le),) * 3, indexing="ij"), axis=-1).reshape(-1, 3) * (0.5 * w)
    cells = list(itertools.product(range(n), repeat=3))
    lim = n * (p + 0.5)
    e = 0.0
    for it, ct in enumerate(cells):
        for js, cs in enumerate(cells):
            ranges = [[ct[a] - cs[a] - n * I for I in range(-p - 2, p + 3) if abs(ct[a] - cs[a] - n * I) <= lim]
                      for a in range(3)]
            for D in itertools.product(*ranges):
                if max(abs(c) for c in D) < 2:
                    continue
                diff = g[:, None, :] - g[None, :, :] + w * np.asarray(D, dtype=np.float64)
                G = kernel_H(np.sqrt(np.sum(diff * diff, axis=-1)), xi)
                e += 0.5 * float(M[it] @ G @ M[js])
    return e


# ---- evaluation --------------------------------------------------------------

def m2l_projector(w: float, L: int, xi: float, rank: int) -> np.ndarray:
    """Low-rank compression of the M2L operators of one level (the SVD
    compression of the far-field operator in the compressed-M2L passage): P =
    U U^T, U = the `rank` leading left singular vectors of the stack [K_d] over
    all 316 offsets d with |d|_inf >= 2.  The compressed operator of offset d
    is P K_d P (the stack is closed under transposition, K_-d = K_d^T, so the
    right singular vectors span the same space)."""
    offs = [d for d in itertools.product(range(-3, 4), repeat=3) if max(abs(c) for c in d) >= 2]
    A = np.hstack([m2l_matrix(d, w, L, xi) for d in offs])
    U = np.linalg.svd(A, full_matrices=False)[0][:, :rank]
    return U @ U.T


# octupoles: stored components (xxx, xxy, xxz, xyy, xyz, xzz, yyy, yyz, yzz, zzz), their derivative orders
# (a, b, c) per axis and their multiplicities in the full symmetric tensor
OMEGA_ABC = [(3, 0, 0), (2, 1, 0), (2, 0, 1), (1, 2, 0), (1, 1, 1), (1, 0, 2), (0, 3, 0), (0, 2, 1), (0, 1, 2),
             (0, 0, 3)]
OMEGA_MULT = [1, 3, 3, 3, 6, 3, 1, 3, 3, 1]


def evaluate(pos, q, mu, theta, edge: float, depth: int, order: int, xi: float, p: int,
             grad: bool = True, nthreads: int = 0, keep: bool = False, root_order: int | None = None,
             m2l_ranks=None, far: str = "fmm", eq_order: int | None = None, leaves: int | None = None,
             omega=None) -> dict:
    """root_order: Chebyshev order of the root grid that carries the far
    images (depth >= 1); defaults to `order`.  m2l_ranks: optional rank per
    level (index e = 1..depth; a rank >= L^3 or 0 leaves the level
    uncompressed) of the compressed M2L operators.  far = "fft": the far
    field of ANKH-FFT instead (leaf level only, equispaced order eq_order;
    the far images are inside its matrix, so e_per = 0); its single-level
    leaf grid may have any number `leaves` of leaves per axis (default 2^depth)."""
    if leaves is not None and far != "fft":
        raise ValueError("a leaf grid that is not an octree level needs far='fft'")
    pos = wrap(_c64(pos, (-1, 3)), edge)
    N = pos.shape[0]
    q = _c64(q, (N,))
    mu = _c64(mu, (N, 3))
    theta = _c64(theta, (N, 6))
    omega = _c64(omega, (N, 10))
    L = order
    nu = L ** 3
    E = depth
    nleaf_ax = (1 << E) if leaves is None else int(leaves)
    w_leaf = edge / nleaf_ax
    h = 0.5 * w_leaf

    # step 1: tree
    ijk = leaf_index(pos, edge, E, nleaf_ax)
    leaf = (ijk[:, 0] * nleaf_ax + ijk[:, 1]) * nleaf_ax + ijk[:, 2]
    ctr = -0.5 * edge + (ijk + 0.5) * w_leaf
    yhat = (pos - ctr) / h

    # step 2: modified charges (Alg. 2), derivatives up to 2 (3 for forces)
    nd = (3 if grad else 2) + (1 if omega is not None else 0)
    S = lagrange_derivs(yhat, L, nd, h)          # [N, 3, nd+1, L]
    Sx, Sy, Sz = S[:, 0], S[:, 1], S[:, 2]

    def tens(a, b, c):
        return np.einsum("ni,nj,nk->nijk", Sx[:, a], Sy[:, b], Sz[:, c])

    contrib = q[:, None, None, None] * tens(0, 0, 0)
    if mu is not None:
        contrib += mu[:, 0, None, None, None] * tens(1, 0, 0)
        contrib += mu[:, 1, None, None, None] * tens(0, 1, 0)
        contrib += mu[:, 2, None, None, None] * tens(0, 0, 1)
    if theta is not None:
        xx, xy, xz, yy, yz, zz = [theta[:, c, None, None, None] for c in range(6)]
        contrib += xx * tens(2, 0, 0) + 2 * xy * tens(1, 1, 0) + 2 * xz * tens(1, 0, 1)
        contrib += yy * tens(0, 2, 0) + 2 * yz * tens(0, 1, 1) + zz * tens(0, 0, 2)
    if omega is not None:
        # Omega : grad^3 S_k, every stored component with its multiplicity
        for c, (a, b, cc) in enumerate(OMEGA_ABC):
            contrib += OMEGA_MULT[c] * omega[:, c, None, None, None] * tens(a, b, cc)
    Q = np.zeros((nleaf_ax ** 3, L, L, L))
    np.add.at(Q, leaf, contrib)

    if far == "fft":
        e_fft, Lam_fft, _ = fft_far(Q.reshape(-1, nu), nleaf_ax, L, int(eq_order),
                                    fft_kernel_table(nleaf_ax, w_leaf, int(eq_order), xi, p))
        e_far_levels, e_per, M, Lloc, Cper = [e_fft], 0.0, None, None, None
    else:
        # upward pass (M2M) to the root
        V = m2m_1d(L)
        L0 = L if (E == 0 or root_order is None) else int(root_order)
        V0 = m2m_1d(L0, L)          # level 1 -> root
        M = [None] * (E + 1)
        M[E] = Q.reshape(nleaf_ax, nleaf_ax, nleaf_ax, nu)
        for e in range(E - 1, -1, -1):
            n = 1 << e
            child = M[e + 1].reshape(n, 2, n, 2, n, 2, L, L, L)
            Vp, Lp = (V0, L0) if e == 0 else (V, L)
            par = np.zeros((n, n, n, Lp, Lp, Lp))
            for bx, by, bz in itertools.product((0, 1), repeat=3):
                par += np.einsum("ai,bj,ck,xyzijk->xyzabc", Vp[bx], Vp[by], Vp[bz],
                                 child[:, bx, :, by, :, bz])
            M[e] = par.reshape(n, n, n, Lp ** 3)

        # far field by M2L on every level 1..E (cells of the adjacent images included)
        offs = interaction_offsets()
        Lloc = [None] * (E + 1)
        e_far_levels = []
        for e in range(1, E + 1):
            n = 1 << e
            w = edge / n
            acc = np.zeros((n, n, n, nu))
            r = 0 if m2l_ranks is None else int(m2l_ranks[e])
            P = m2l_projector(w, L, xi, r) if 0 < r < nu else None
            for d in offs:
                K = m2l_matrix(d, w, L, xi)
                if P is not None:
                    K = P @ K @ P
                Ms = np.roll(M[e], shift=(-d[0], -d[1], -d[2]), axis=(0, 1, 2))
                acc += _valid_mask(n, d)[..., None] * (Ms @ K.T)
            Lloc[e] = acc
            e_far_levels.append(0.5 * float(np.sum(M[e] * acc)))

        # far periodic images through the root
        nu0 = L0 ** 3
        Cper = periodic_root_matrix(edge, L0, xi, p)
        Lroot = M[0].reshape(nu0) @ Cper.T
        e_per = 0.5 * float(M[0].reshape(nu0) @ Lroot)

    # near field: direct pair sums over adjacent leaves
    eatom = np.zeros(N)
    Fn = np.zeros((N, 3)) if grad else None
    Gn = np.zeros((N, 3)) if grad else None
    rc = _oracle_lib().oracle_near_field_o3(N, _p(pos), _p(q), _p(mu), _p(theta), _p(omega), float(edge),
                                            float(xi), int(nleaf_ax), int(nthreads), _p(eatom), _p(Fn), _p(Gn))
    if rc != 0:
        raise ValueError("oracle_near_field failed")
    e_near = float(np.sum(eatom))

    # self energy and background
    s = q * q
    if mu is not None:
        s = s + (2 * xi ** 2 / 3) * np.sum(mu * mu, axis=1)
    if theta is not None:
        tt = theta[:, 0] ** 2 + theta[:, 3] ** 2 + theta[:, 5] ** 2 + 2 * (
            theta[:, 1] ** 2 + theta[:, 2] ** 2 + theta[:, 4] ** 2)
        s = s + (8 * xi ** 4 / 5) * tt
    if omega is not None:
        oo = np.sum(np.array(OMEGA_MULT)[None, :] * omega ** 2, axis=1)      # Omega : Omega
        s = s + (48 * xi ** 6 / 7) * oo
    e_self = float(-(xi / math.sqrt(math.pi)) * np.sum(s))
    Qtot = float(np.sum(q))
    e_bg = -math.pi * Qtot ** 2 / (2 * edge ** 3 * xi ** 2)

    out = dict(energy=e_near + sum(e_far_levels) + e_per + e_self + e_bg, e_near=e_near,
               e_far_levels=e_far_levels, e_per=e_per, e_self=e_self, e_bg=e_bg)

    if grad:
        # leaf local expansions: from the transform (ANKH-FFT), or by the downward pass (L2L = M2M^T)
        if far == "fft":
            Lam = Lam_fft
        else:
            Lam = Lroot.reshape(1, 1, 1, nu0)
            for e in range(1, E + 1):
                n = 1 << e
                down = np.zeros((n, n, n, L, L, L))
                Vp, Lp = (V0, L0) if e == 1 else (V, L)
                par = Lam.reshape(n // 2, n // 2, n // 2, Lp, Lp, Lp)
                dv = down.reshape(n // 2, 2, n // 2, 2, n // 2, 2, L, L, L)
                for bx, by, bz in itertools.product((0, 1), repeat=3):
                    dv[:, bx, :, by, :, bz] += np.einsum("ai,bj,ck,xyzabc->xyzijk", Vp[bx], Vp[by], Vp[bz], par)
                Lam = down.reshape(n, n, n, nu) + Lloc[e]
        Lam_leaf = Lam.reshape(-1, L, L, L)[leaf]          # [N, L, L, L]
        # L2P: derivatives of phi(y) = sum_k Lam_k S_k(y) up to order 3 (4 with octupoles)
        phi = {}
        for a in range(nd + 1):
            for b in range(nd + 1 - a):
                for c in range(nd + 1 - a - b):
                    phi[(a, b, c)] = np.einsum("nijk,ni,nj,nk->n", Lam_leaf, Sx[:, a], Sy[:, b], Sz[:, c])

        def dphi(*axes):
            cnt = [0, 0, 0]
            for ax in axes:
                cnt[ax] += 1
            return phi[tuple(cnt)]

        Ff = np.zeros((N, 3))
        Gf = np.zeros((N, 3))
        Th = None
        if theta is not None:
            t = theta
            Th = np.stack([np.stack([t[:, 0], t[:, 1], t[:, 2]], 1),
                           np.stack([t[:, 1], t[:, 3], t[:, 4]], 1),
                           np.stack([t[:, 2], t[:, 4], t[:, 5]], 1)], 1)
        for x in range(3):
            g = q * dphi(x)
            if mu is not None:
                for a in range(3):
                    g = g + mu[:, a] * dphi(a, x)
            if Th is not None:
                for a in range(3):
                    for b in range(3):
                        g = g + Th[:, a, b] * dphi(a, b, x)
            if omega is not None:
                for c, (a, b, cc) in enumerate(OMEGA_ABC):
                    cnt = [a, b, cc]
                    cnt[x] += 1
                    g = g + OMEGA_MULT[c] * omega[:, c] * phi[tuple(cnt)]
            Ff[:, x] = -g
            Gf[:, x] = dphi(x)
        # equals sum(e_far_levels) + e_per: the leaf form of the same quadratic form
        e_far_leaf = 0.5 * float(np.sum(Q.reshape(-1, nu) * Lam.reshape(-1, nu)))
        Gs = np.zeros((N, 3)) if mu is None else -(4 * xi ** 3 / (3 * math.sqrt(math.pi))) * mu
        out.update(forces=Fn + Ff, dEdmu=(Gn + Gf + Gs) if mu is not None else np.zeros((N, 3)),
                   forces_near=Fn, forces_far=Ff, e_far_leaf=e_far_leaf)
    if keep:
        out.update(Q=Q, M=M, Lloc=Lloc, leaf=leaf, Cper=Cper, Lam=Lam if grad else None)
    return out
