"""FP64 CPU oracle for the AO -> MO value/gradient/Laplacian path (test
infrastructure only).

Only the tests, the smoke check and the benchmark's CPU-baseline leg import
this package.  The library never does; the two share no code.  The arithmetic
lives in ``oracle.c`` (plain C, FP64, no BLAS); this module builds it with gcc
and marshals numpy arrays through ctypes.

Layouts (C order): AO and MO results are ``[point][component][function]`` with
components (value, d/dx, d/dy, d/dz, Laplacian); with ``nq=14`` the AO result
also carries the Hessian (xx xy xz yy yz zz) and the gradient of the
Laplacian (components 5..13).  MO values alone and the electron density of a
determinant (Section 5.4, orbital visualisation) are taken from the value rows.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
NQ_FULL = 14

_lib = None


def build(force: bool = True) -> str:
    """Compile oracle.c into liboracle.so (gcc, -O2, OpenMP, no fast-math)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared",
                               "-fno-fast-math", "-ffp-contract=off", _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        _load_from(ctypes.CDLL(_LIB))
    return _lib


def use_library(path: Optional[str]):
    """Load the oracle's arithmetic from another build of oracle.c (the
    mutation tests plant mistakes in copies); None restores the default."""
    global _lib
    _lib = None
    if path is None:
        return _load()
    lib = ctypes.CDLL(path)
    global _LIB
    saved = _LIB
    try:
        _LIB = path
        _lib = None
        return _load_from(lib)
    finally:
        _LIB = saved


def _load_from(lib):
    global _lib
    P = ctypes.c_void_p
    I64 = ctypes.c_int64
    lib.oracle_ao_num.argtypes = [I64, P]
    lib.oracle_ao_num.restype = I64
    lib.oracle_normalisation.argtypes = [I64, P, P, P, P, P, P, P]
    lib.oracle_normalisation.restype = None
    lib.oracle_ao_derivs.argtypes = [I64, P, I64, P, P, P, P, P, I64, P, ctypes.c_double,
                                     ctypes.c_int, P]
    lib.oracle_ao_derivs.restype = ctypes.c_int
    lib.oracle_mo_vgl.argtypes = [I64, I64, I64, P, P, P]
    lib.oracle_mo_vgl.restype = ctypes.c_int
    lib.oracle_adjoint.argtypes = [I64, P, I64, P, P, P, P, P, I64, P, ctypes.c_double,
                                   I64, P, P, P, P, P, P, P, P]
    lib.oracle_adjoint.restype = ctypes.c_int
    _lib = lib
    return lib


def _c(a, dtype):
    return np.ascontiguousarray(a, dtype=dtype)


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


class _Basis:
    def __init__(self, s):
        self.nucl = _c(s.nucl_coord, np.float64)
        self.sn = _c(s.shell_nucleus, np.int64)
        self.sl = _c(s.shell_ang_mom, np.int32)
        self.so = _c(s.shell_prim_offset, np.int64)
        self.ex = _c(s.exponent, np.float64)
        self.co = _c(s.coefficient, np.float64)
        self.ao_num = int(_load().oracle_ao_num(self.sl.shape[0], _ptr(self.sl)))

    def args(self):
        return (self.nucl.shape[0], _ptr(self.nucl), self.sl.shape[0], _ptr(self.sn), _ptr(self.sl),
                _ptr(self.so), _ptr(self.ex), _ptr(self.co))


def normalisation(sys_):
    """(prim_factor f, shell_factor N_s, ao_factor M) as the oracle derives them."""
    b = _Basis(sys_)
    f = np.empty(b.ex.shape[0])
    ns = np.empty(b.sl.shape[0])
    m = np.empty(b.ao_num)
    _load().oracle_normalisation(b.sl.shape[0], _ptr(b.sl), _ptr(b.so), _ptr(b.ex), _ptr(b.co),
                                 _ptr(f), _ptr(ns), _ptr(m))
    return f, ns, m


def ao_derivs(sys_, points: np.ndarray, B: float = 53.0, nq: int = 5) -> np.ndarray:
    """AO quantities at `points` [P,3]: returns [P, nq, ao_num] (nq = 5 or 14).
    B <= 0 disables the exponent cutoff."""
    b = _Basis(sys_)
    pts = _c(points, np.float64).reshape(-1, 3)
    out = np.empty((pts.shape[0], nq, b.ao_num))
    rc = _load().oracle_ao_derivs(*b.args(), pts.shape[0], _ptr(pts), float(B), int(nq), _ptr(out))
    if rc:
        raise RuntimeError(f"oracle_ao_derivs failed ({rc})")
    return out


def ao_vgl(sys_, points: Optional[np.ndarray] = None, B: float = 53.0) -> np.ndarray:
    """AO value/gradient/Laplacian [P, 5, ao_num] (default points: all walkers)."""
    return ao_derivs(sys_, sys_.points() if points is None else points, B, 5)


def mo_vgl_from_ao(ao: np.ndarray, coef: np.ndarray) -> np.ndarray:
    ao = _c(ao, np.float64)
    coef = _c(coef, np.float64)
    P, five, K = ao.shape
    N = coef.shape[0]
    assert five == 5 and coef.shape[1] == K
    out = np.empty((P, 5, N))
    _load().oracle_mo_vgl(P, K, N, _ptr(ao), _ptr(coef), _ptr(out))
    return out


def mo_vgl(sys_, points: Optional[np.ndarray] = None, B: float = 53.0,
           coef: Optional[np.ndarray] = None) -> np.ndarray:
    """mo_vgl [P, 5, mo_num] at `points` (default: every walker's electrons)."""
    ao = ao_vgl(sys_, points, B)
    return mo_vgl_from_ao(ao, sys_.mo_coef if coef is None else coef)


def adjoint(sys_, w: np.ndarray, points: Optional[np.ndarray] = None, B: float = 53.0,
            coef: Optional[np.ndarray] = None, nucl: Optional[np.ndarray] = None,
            with_abs: bool = True):
    """Gradients of sum(W * mo_vgl): returns dict with d_coef [mo, ao],
    d_elec [P, 3], d_nucl [nucl, 3] and the matching *_abs sums."""
    import copy
    s = sys_
    if nucl is not None:
        s = copy.copy(sys_)
        s.nucl_coord = nucl
    b = _Basis(s)
    pts = _c(sys_.points() if points is None else points, np.float64).reshape(-1, 3)
    C = _c(sys_.mo_coef if coef is None else coef, np.float64)
    N = C.shape[0]
    W = _c(w, np.float64).reshape(pts.shape[0], 5, N)
    out = {
        "d_coef": np.empty((N, b.ao_num)),
        "d_elec": np.empty((pts.shape[0], 3)),
        "d_nucl": np.empty((b.nucl.shape[0], 3)),
    }
    if with_abs:
        out.update({"d_coef_abs": np.empty((N, b.ao_num)), "d_elec_abs": np.empty((pts.shape[0], 3)),
                    "d_nucl_abs": np.empty((b.nucl.shape[0], 3))})
    rc = _load().oracle_adjoint(*b.args(), pts.shape[0], _ptr(pts), float(B), N, _ptr(C), _ptr(W),
                                _ptr(out["d_coef"]), _ptr(out["d_elec"]), _ptr(out["d_nucl"]),
                                _ptr(out.get("d_coef_abs")), _ptr(out.get("d_elec_abs")),
                                _ptr(out.get("d_nucl_abs")))
    if rc:
        raise RuntimeError(f"oracle_adjoint failed ({rc})")
    return out


def _ao_nucleus(sys_) -> np.ndarray:
    """Nucleus index of every AO (AOs numbered shell by shell)."""
    return np.repeat(np.asarray(sys_.shell_nucleus, dtype=np.int64),
                     [(int(l) + 1) * (int(l) + 2) // 2 for l in sys_.shell_ang_mom])


# (i, j) -> AO derivative quantity of the Hessian component d_i d_j chi
_HESS_Q = ((5, 6, 7), (6, 8, 9), (7, 9, 10))


def adjoint_products(sys_, w: np.ndarray, points: Optional[np.ndarray] = None, B: float = 53.0,
                     coef: Optional[np.ndarray] = None, with_mo: bool = False,
                     chunk: Optional[int] = None):
    """The gradients of `adjoint` (same definitions, same dict keys with the
    *_abs sums), for workloads too large for its literal loops.

    The two sums over an index that runs over thousands of values are taken
    as matrix products with numpy (a library step), chunk by chunk of points,
    on the oracle's AO derivatives up to third order:
      Gbar[p,c,:] = W[p,c,:] C            (sum over MOs)
      dC         += W_chunk^T ao_chunk    (sum over points and components)
    and the electron and nuclear terms follow the definitions of `adjoint`:
      t[p,k,i] = Gbar[p,0,k] d_i chi_k + sum_j Gbar[p,1+j,k] d_i d_j chi_k
                 + Gbar[p,4,k] d_i lap chi_k,
      dR_elec[p,i] = sum_k t[p,k,i],  dR_nucl[A,i] = -sum_p sum_{k on A} t[p,k,i].
    With with_mo, also returns "mo" [P, 5, mo] = ao C^T (Section 3.2)."""
    pts = _c(sys_.points() if points is None else points, np.float64).reshape(-1, 3)
    C = _c(sys_.mo_coef if coef is None else coef, np.float64)
    N, K = C.shape
    P = pts.shape[0]
    W = np.asarray(w, dtype=np.float64).reshape(P, 5, N)
    if chunk is None:  # keep one chunk's AO derivatives near 512 MB
        chunk = max(16, int(512e6 // (NQ_FULL * K * 8)))
    own = _ao_nucleus(sys_)
    n_nucl = int(np.asarray(sys_.nucl_coord).reshape(-1, 3).shape[0])
    out = {"d_coef": np.zeros((N, K)), "d_coef_abs": np.zeros((N, K)),
           "d_elec": np.empty((P, 3)), "d_elec_abs": np.empty((P, 3)),
           "d_nucl": np.zeros((n_nucl, 3)), "d_nucl_abs": np.zeros((n_nucl, 3))}
    if with_mo:
        out["mo"] = np.empty((P, 5, N))
    for a in range(0, P, chunk):
        b = min(a + chunk, P)
        ao = ao_derivs(sys_, pts[a:b], B, NQ_FULL)          # [c, 14, K]
        Wc = W[a:b]                                         # [c, 5, N]
        gbar = np.matmul(Wc, C)                             # [c, 5, K]
        for i in range(3):
            terms = [gbar[:, 0] * ao[:, 1 + i]] + \
                    [gbar[:, 1 + j] * ao[:, _HESS_Q[i][j]] for j in range(3)] + \
                    [gbar[:, 4] * ao[:, 11 + i]]
            t = terms[0] + terms[1] + terms[2] + terms[3] + terms[4]           # [c, K]
            ta = (np.abs(terms[0]) + np.abs(terms[1]) + np.abs(terms[2]) + np.abs(terms[3])
                  + np.abs(terms[4]))
            out["d_elec"][a:b, i] = t.sum(axis=1)
            out["d_elec_abs"][a:b, i] = ta.sum(axis=1)
            np.subtract.at(out["d_nucl"][:, i], own, t.sum(axis=0))
            np.add.at(out["d_nucl_abs"][:, i], own, ta.sum(axis=0))
        a5 = np.ascontiguousarray(ao[:, :5]).reshape(-1, K)  # rows (point, component)
        w5 = Wc.reshape(-1, N)
        out["d_coef"] += w5.T @ a5
        out["d_coef_abs"] += np.abs(w5).T @ np.abs(a5)
        if with_mo:
            out["mo"][a:b] = (a5 @ C.T).reshape(b - a, 5, N)
    return out


def mo_value(sys_, points: Optional[np.ndarray] = None, B: float = 53.0,
             coef: Optional[np.ndarray] = None) -> np.ndarray:
    """MO values [P, mo] (the value rows of mo_vgl)."""
    return mo_vgl(sys_, points, B, coef)[:, 0, :]


def density(sys_, occ: np.ndarray, points: Optional[np.ndarray] = None, B: float = 53.0,
            coef: Optional[np.ndarray] = None, with_abs: bool = False):
    """Electron density of a determinant, rho(r) = sum_n occ[n] phi_n(r)^2
    (Section 5.4: density as a sum of squared MOs), at `points` (default: all
    walkers).  With with_abs, also returns sum_n |occ[n]| (sum_k |C_nk chi_k|)^2,
    an upper scale of the rounding error of any evaluation of rho."""
    C = np.asarray(sys_.mo_coef if coef is None else coef, dtype=np.float64)
    occ = np.asarray(occ, dtype=np.float64).reshape(-1)
    assert occ.shape[0] == C.shape[0]
    keep = occ != 0.0
    pts = np.asarray(sys_.points() if points is None else points, dtype=np.float64).reshape(-1, 3)
    rho = np.zeros(pts.shape[0])
    rho_abs = np.zeros(pts.shape[0])
    if keep.any():
        for a in range(0, pts.shape[0], 16384):  # bounded memory: points in chunks
            b = min(a + 16384, pts.shape[0])
            ao = ao_vgl(sys_, pts[a:b], B)[:, 0, :]       # [chunk, ao]
            phi = ao @ C[keep].T                          # [chunk, n_occ]
            rho[a:b] = (phi * phi) @ occ[keep]
            if with_abs:
                phi_abs = np.abs(ao) @ np.abs(C[keep]).T
                rho_abs[a:b] = (phi_abs * phi_abs) @ np.abs(occ[keep])
    return (rho, rho_abs) if with_abs else rho


def _s_ao_columns(sys_, nucleus: int) -> np.ndarray:
    """AO indices of the s-type shells on `nucleus` (AOs numbered shell by
    shell, (l+1)(l+2)/2 Cartesian functions each)."""
    cols, k = [], 0
    for sh, (A, l) in enumerate(zip(sys_.shell_nucleus, sys_.shell_ang_mom)):
        if int(A) == nucleus and int(l) == 0:
            cols.append(k)
        k += (int(l) + 1) * (int(l) + 2) // 2
    return np.asarray(cols, dtype=np.int64)


def cusp_coefficients(sys_, charge, r_cusp, B: float = 53.0, coef: Optional[np.ndarray] = None):
    """Coefficients f[A] of shape [mo, 4] of the cusp polynomial of every
    nucleus with r_cusp[A] > 0 (Section 3.3), as a dict A -> f.

    With r = |r - R_A|, R = r_cusp[A], Z = charge[A] and phi^s the part of MO i
    carried by the s-type AOs on A, p(r) = sum_k f_k r^k satisfies
      p(R) = phi^s(R),  p'(R) = phi^s'(R),  p''(R) = phi^s''(R)  (continuity
      of the value and of the first two radial derivatives at R), and
      p'(0) = -Z (phi(R_A) - phi^s(R_A) + p(0))  (the electron-nucleus cusp of
      the corrected orbital).
    The radial derivatives of phi^s at R are read off the oracle's gradient
    and Laplacian at R_A + R e_x: phi^s' = d/dx, phi^s'' = lap - 2 phi^s' / R."""
    C = np.asarray(sys_.mo_coef if coef is None else coef, dtype=np.float64)
    out = {}
    for A in range(sys_.nucl_num):
        R = float(r_cusp[A])
        if R <= 0.0:
            continue
        Z = float(charge[A])
        cols = _s_ao_columns(sys_, A)
        Cs = C[:, cols]
        centre = sys_.nucl_coord[A]
        at_nuc = ao_vgl(sys_, centre[None, :], B)[0]                  # [5, ao]
        delta = C @ at_nuc[0] - Cs @ at_nuc[0, cols]                  # phi(R_A) - phi^s(R_A)
        on_sphere = ao_vgl(sys_, (centre + np.array([R, 0.0, 0.0]))[None, :], B)[0]
        v = Cs @ on_sphere[0, cols]
        v1 = Cs @ on_sphere[1, cols]
        v2 = Cs @ on_sphere[4, cols] - 2.0 * v1 / R
        M = np.array([[1.0, R, R * R, R ** 3],
                      [0.0, 1.0, 2.0 * R, 3.0 * R * R],
                      [0.0, 0.0, 2.0, 6.0 * R],
                      [Z, 1.0, 0.0, 0.0]])
        rhs = np.stack([v, v1, v2, -Z * delta])                       # [4, mo]
        out[A] = np.linalg.solve(M, rhs).T                            # [mo, 4]
    return out


def mo_vgl_cusp(sys_, charge, r_cusp, points: Optional[np.ndarray] = None, B: float = 53.0,
                coef: Optional[np.ndarray] = None) -> np.ndarray:
    """Cusp-corrected mo_vgl [P, 5, mo] (Section 3.3): inside the sphere of
    radius r_cusp[A] around nucleus A, phi_i - phi_i^{s_A} + sum_k f_k r^k,
    with value, gradient and Laplacian of the radial polynomial
    (p, p'(r) d/r, p'' + 2 p'/r) and of phi^{s_A} from the oracle's AOs."""
    C = np.asarray(sys_.mo_coef if coef is None else coef, dtype=np.float64)
    pts = np.asarray(sys_.points() if points is None else points, dtype=np.float64).reshape(-1, 3)
    ao = ao_vgl(sys_, pts, B)                                         # [P, 5, ao]
    mo = np.einsum("pck,nk->pcn", ao, C)
    for A, f in cusp_coefficients(sys_, charge, r_cusp, B, C).items():
        d = pts - sys_.nucl_coord[A]
        r = np.sqrt(np.sum(d * d, axis=1))
        inside = np.nonzero(r < float(r_cusp[A]))[0]
        if inside.size == 0:
            continue
        cols = _s_ao_columns(sys_, A)
        phis = np.einsum("pck,nk->pcn", ao[inside][:, :, cols], C[:, cols])
        ri = r[inside][:, None]
        p0 = f[:, 0] + ri * (f[:, 1] + ri * (f[:, 2] + ri * f[:, 3]))
        p1 = f[:, 1] + ri * (2.0 * f[:, 2] + 3.0 * ri * f[:, 3])
        p2 = 2.0 * f[:, 2] + 6.0 * ri * f[:, 3]
        poly = np.empty_like(phis)
        poly[:, 0] = p0
        with np.errstate(divide="ignore", invalid="ignore"):  # r = 0: the cusp diverges
            poly[:, 1:4] = (p1 / ri)[:, None, :] * d[inside][:, :, None]
            poly[:, 4] = p2 + 2.0 * p1 / ri
        mo[inside] += poly - phis
    return mo


def det_adj(a: np.ndarray):
    """Determinant and adjugate of every matrix of a [..., n, n] (Section 3.4:
    adj(A) is the transpose of the cofactor matrix, A^-1 = adj(A) / det(A)).
    The adjugate follows the definition: adj_ji = (-1)^(i+j) times the
    determinant of A without row i and column j.  Determinants come from
    numpy's LU routine (a library step)."""
    a = np.asarray(a, dtype=np.float64)
    n = a.shape[-1]
    flat = a.reshape(-1, n, n)
    det = np.linalg.det(flat)
    adj = np.empty_like(flat)
    if n == 1:
        adj[:] = 1.0
    else:
        for i in range(n):
            for j in range(n):
                minor = np.delete(np.delete(flat, i, axis=1), j, axis=2)
                adj[:, j, i] = (-1.0) ** (i + j) * np.linalg.det(minor)
    return det.reshape(a.shape[:-2]), adj.reshape(a.shape)


def een_terms(nord: int):
    """(p, k, l) of the three-body Jastrow terms in the order of the
    coefficient array (Section 3.5): p = 2..nord, k = 0..p-1,
    l = 0..p-k-2*delta(k,0), each ascending, keeping the terms with p-k-l
    even (so that (p-k-l)/2 is a whole power)."""
    out = []
    for p in range(2, nord + 1):
        for k in range(0, p):
            for l in range(0, p - k - (2 if k == 0 else 0) + 1):
                if (p - k - l) % 2 == 0:
                    out.append((p, k, l))
    return out


def jastrow_een(elec: np.ndarray, nucl: np.ndarray, kappa: float, nord: int, c: np.ndarray) -> np.ndarray:
    """Three-body (electron-electron-nucleus) Jastrow factor of every walker
    by its original pairwise definition (Section 3.5):
      J = sum_a sum_{i>j} sum_{(p,k,l)} c[t, a] rt_ij^k (Rt_ia^l + Rt_ja^l) (Rt_ia Rt_ja)^((p-k-l)/2)
    with rt_ij = exp(-kappa r_ij), Rt_ia = exp(-kappa |r_i - R_a|).
    elec [walk, elec, 3], nucl [nucl, 3], c [n_terms, nucl] (een_terms order).
    Returns J [walk]."""
    elec = np.asarray(elec, dtype=np.float64)
    nucl = np.asarray(nucl, dtype=np.float64)
    c = np.asarray(c, dtype=np.float64)
    terms = een_terms(nord)
    assert c.shape == (len(terms), nucl.shape[0])
    W, ne = elec.shape[0], elec.shape[1]
    iu, ju = np.triu_indices(ne, k=1)                      # pairs i < j (the sum is symmetric)
    out = np.zeros(W)
    for w in range(W):
        x = elec[w]
        r = np.linalg.norm(x[iu] - x[ju], axis=1)          # [pairs]
        rt = np.exp(-kappa * r)
        R = np.linalg.norm(x[:, None, :] - nucl[None, :, :], axis=2)  # [elec, nucl]
        Rt = np.exp(-kappa * R)
        Ri, Rj = Rt[iu], Rt[ju]                            # [pairs, nucl]
        total = 0.0
        for t, (p, k, l) in enumerate(terms):
            m = (p - k - l) // 2
            val = (rt ** k)[:, None] * (Ri ** l + Rj ** l) * (Ri * Rj) ** m   # [pairs, nucl]
            total += float(np.sum(val.sum(axis=0) * c[t]))
        out[w] = total
    return out
