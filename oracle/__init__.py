"""Plain CPU oracle for the ParO plane-wave hot path (test infrastructure).

Only the tests, the smoke check and the CPU-baseline leg of the benchmark may
import this package.  It wraps ``paro_oracle.c`` (plain C, OpenMP over
bands, radix-2 FFT on a power-of-two padded grid, cyclic Jacobi eigensolver)
through ctypes and shares no code with the GPU library.

Layouts: orbital blocks are (bands, n_g) complex128 numpy arrays, band-major;
small dense matrices are returned as ordinary numpy (row-major) arrays.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liboracle.so")
SRC_PATH = os.path.join(_HERE, "paro_oracle.c")

F_NEGCURV, F_CHOL, F_NAN = 1, 2, 4


# -march=x86-64-v3 (AVX2 + FMA) rather than -march=native: the library is
# built once and may run on a host with another CPU model.
CFLAGS = ["-O3", "-march=x86-64-v3", "-fopenmp", "-std=gnu11"]


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (CFLAGS, OpenMP)."""
    if force or not os.path.exists(LIB_PATH) or \
            os.path.getmtime(LIB_PATH) < os.path.getmtime(SRC_PATH):
        tmp = LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", *CFLAGS, "-shared", "-fPIC",
                               SRC_PATH, "-o", tmp, "-lm"])
        os.replace(tmp, LIB_PATH)
    return LIB_PATH


_lib = None

_dp = C.POINTER(C.c_double)
_ip = C.POINTER(C.c_int32)
_vp = C.c_void_p


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        build()
    lib = C.CDLL(LIB_PATH)
    sig = {
        "orc_sphere": (C.c_int64, [_dp, C.c_double, _ip, C.c_int64, _ip]),
        "orc_ham_create": (C.c_int32, [_dp, C.c_double, _ip, _dp, C.c_int32, _dp, _ip, _ip,
                                       _dp, _dp, C.POINTER(_vp)]),
        "orc_ham_destroy": (None, [_vp]),
        "orc_ham_ng": (C.c_int64, [_vp]),
        "orc_ham_info": (None, [_vp, _ip, _ip]),
        "orc_ham_miller": (None, [_vp, _ip]),
        "orc_ham_kin": (None, [_vp, _dp]),
        "orc_ham_beta": (None, [_vp, _vp]),
        "orc_ham_vmin": (C.c_double, [_vp]),
        "orc_vtilde": (None, [_ip, _dp, _ip, _vp]),
        "orc_fft1d": (None, [_vp, C.c_int32, C.c_int32]),
        "orc_fft3d": (None, [_vp, _ip, C.c_int32]),
        "orc_apply_h": (None, [_vp, C.c_int32, _vp, _dp, _vp]),
        "orc_dense_h": (None, [_vp, _vp]),
        "orc_heev": (C.c_int32, [C.c_int32, _vp, _dp, _vp]),
        "orc_cholesky": (C.c_int32, [C.c_int32, _vp]),
        "orc_rayleigh_ritz": (C.c_int32, [C.c_int64, C.c_int32, C.c_int32, _vp, _vp, _dp, _vp, _vp]),
        "orc_teter": (C.c_double, [C.c_double]),
        "orc_pcg": (C.c_int32, [_vp, C.c_int32, _vp, _vp, _dp, _dp, C.c_int32, C.c_int32, _vp, _ip, _dp]),
        "orc_nl_min_eig": (C.c_double, [_vp]),
        "orc_shift_bound": (C.c_double, [_vp]),
        "orc_paro": (C.c_int32, [_vp, C.c_int32, _vp, _vp, _dp, C.c_int32, C.c_int32, C.c_int32,
                                 C.c_int32, C.c_double, _dp, _dp, _dp]),
        "orc_num_threads": (C.c_int32, []),
        "orc_residual_norms": (None, [C.c_int64, C.c_int32, _vp, _vp, _dp, _dp]),
        "orc_density": (None, [_vp, C.c_int32, _vp, _dp, _dp]),
        "orc_projector_gradient": (None, [_vp, C.c_int32, _vp, _dp, _dp, _dp]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def _d(a):
    return a.ctypes.data_as(_dp)


def _i(a):
    return a.ctypes.data_as(_ip)


def _v(a):
    return C.c_void_p(a.ctypes.data)


def _cd(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _cc(a):
    return np.ascontiguousarray(a, dtype=np.complex128)


def num_threads() -> int:
    return int(_load().orc_num_threads())


def sphere(cell, ecut):
    """Miller indices (n_g x 3, lexicographic) of the cutoff sphere (e3), and n_max."""
    lib = _load()
    cell = _cd(cell).reshape(9)
    nmax = np.zeros(3, np.int32)
    n = lib.orc_sphere(_d(cell), float(ecut), None, 0, _i(nmax))
    mil = np.zeros((n, 3), np.int32)
    lib.orc_sphere(_d(cell), float(ecut), _i(mil), n, _i(nmax))
    return mil, nmax


def vtilde(vloc, K):
    """Direct-DFT Fourier coefficients Vt(k), |k_d| <= K_d, shape (2K+1)^3."""
    lib = _load()
    v = _cd(vloc)
    grid = np.array(v.shape, np.int32)
    K = np.array(K, np.int32)
    out = np.zeros(tuple(2 * K + 1), np.complex128)
    lib.orc_vtilde(_i(grid), _d(v), _i(K), _v(out))
    return out


def fft1d(x, sign):
    y = _cc(x).copy()
    _load().orc_fft1d(_v(y), y.size, int(sign))
    return y


def fft3d(x, sign):
    y = _cc(x).copy()
    M = np.array(y.shape, np.int32)
    _load().orc_fft3d(_v(y), _i(M), int(sign))
    return y


def heev(A):
    """Ascending eigenvalues and eigenvectors of a Hermitian matrix (Jacobi)."""
    A = np.asarray(A, np.complex128)
    n = A.shape[0]
    buf = _cc(A.T)  # column-major
    w = np.zeros(n)
    V = np.zeros((n, n), np.complex128)
    sweeps = _load().orc_heev(n, _v(buf), _d(w), _v(V))
    return w, V.T.copy(), sweeps


def cholesky(A):
    A = np.asarray(A, np.complex128)
    n = A.shape[0]
    buf = _cc(A.T)
    rc = _load().orc_cholesky(n, _v(buf))
    return rc, buf.T.copy()


def teter(x):
    return _load().orc_teter(float(x))


def residual_norms(psi, hpsi, eps):
    """|hpsi_b - eps_b psi_b| per band (bands x n_g blocks)."""
    psi, hpsi = _cc(psi), _cc(hpsi)
    nb, ng = psi.shape
    eps = _cd(eps)
    res = np.zeros(nb)
    _load().orc_residual_norms(ng, nb, _v(psi), _v(hpsi), _d(eps), _d(res))
    return res


def rayleigh_ritz(U, W, nkeep):
    """RR on span of the rows of U (bands x n_g); W = H U.  Returns (eps, psi, hpsi, flags)."""
    U = _cc(U)
    W = _cc(W)
    m, ng = U.shape
    eps = np.zeros(nkeep)
    psi = np.zeros((nkeep, ng), np.complex128)
    hpsi = np.zeros((nkeep, ng), np.complex128)
    f = _load().orc_rayleigh_ritz(ng, m, nkeep, _v(U), _v(W), _d(eps), _v(psi), _v(hpsi))
    return eps, psi, hpsi, f


class Hamiltonian:
    """Fixed-potential plane-wave Hamiltonian (e5) held by the oracle."""

    def __init__(self, cell, ecut, vloc, projectors=()):
        lib = _load()
        self._lib = lib
        cell = _cd(cell).reshape(9)
        v = _cd(vloc)
        grid = np.array(v.shape, np.int32)
        npj = len(projectors)
        cen = np.zeros((max(npj, 1), 3))
        pl = np.zeros(max(npj, 1), np.int32)
        pm = np.zeros(max(npj, 1), np.int32)
        pw = np.zeros(max(npj, 1))
        pd = np.zeros(max(npj, 1))
        for i, p in enumerate(projectors):
            cen[i] = p["center"]
            pl[i], pm[i], pw[i], pd[i] = p["l"], p["m"], p["width"], p["d"]
        h = C.c_void_p()
        rc = lib.orc_ham_create(_d(cell), float(ecut), _i(grid), _d(v), npj, _d(cen), _i(pl), _i(pm),
                                _d(pw), _d(pd), C.byref(h))
        if rc != 0:
            raise ValueError(f"oracle: grid {tuple(grid)} too small for the sphere (rc={rc})")
        self._h = h
        self.ng = int(lib.orc_ham_ng(h))
        self.nproj = npj
        nmax = np.zeros(3, np.int32)
        M = np.zeros(3, np.int32)
        lib.orc_ham_info(h, _i(nmax), _i(M))
        self.nmax, self.padded = nmax, M
        self.grid = tuple(int(g) for g in grid)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            self._lib.orc_ham_destroy(h)
            self._h = None

    @property
    def miller(self):
        out = np.zeros((self.ng, 3), np.int32)
        self._lib.orc_ham_miller(self._h, _i(out))
        return out

    @property
    def kin(self):
        out = np.zeros(self.ng)
        self._lib.orc_ham_kin(self._h, _d(out))
        return out

    @property
    def beta(self):
        out = np.zeros((self.nproj, self.ng), np.complex128)
        if self.nproj:
            self._lib.orc_ham_beta(self._h, _v(out))
        return out

    @property
    def vmin(self):
        return float(self._lib.orc_ham_vmin(self._h))

    def apply(self, psi, shift=None):
        psi = _cc(np.atleast_2d(psi))
        nb = psi.shape[0]
        out = np.zeros_like(psi)
        sh = None if shift is None else _cd(np.broadcast_to(np.asarray(shift, np.float64), (nb,)))
        self._lib.orc_apply_h(self._h, nb, _v(psi), None if sh is None else _d(sh), _v(out))
        return out

    def dense(self):
        H = np.zeros((self.ng, self.ng), np.complex128)
        self._lib.orc_dense_h(self._h, _v(H))
        return H.T.copy()  # column-major buffer -> (m, n) array

    def nl_min_eig(self):
        return float(self._lib.orc_nl_min_eig(self._h))

    def shift_bound(self):
        return float(self._lib.orc_shift_bound(self._h))

    def pcg(self, psi, hpsi, eps, shift, ncg, gamma_hist=False, correction=False, projected=False):
        """n_cg PCG steps per band: the source problem of Algorithm 1 (from u = psi), the
        correction equation of Algorithm 2 (correction=True, from e = 0) or the projected
        correction equation of Algorithm 3 (projected=True).  Returns (u or e, flags)."""
        psi, hpsi = _cc(psi), _cc(hpsi)
        nb = psi.shape[0]
        eps = _cd(eps)
        sh = _cd(np.broadcast_to(np.asarray(shift, np.float64), (nb,)))
        u = np.zeros_like(psi)
        flags = np.zeros(nb, np.int32)
        gh = np.zeros((nb, ncg + 1)) if gamma_hist else None
        mode = 2 if projected else int(bool(correction))
        self._lib.orc_pcg(self._h, nb, _v(psi), _v(hpsi), _d(eps), _d(sh), ncg, mode, _v(u), _i(flags),
                          None if gh is None else _d(gh))
        return (u, flags, gh) if gamma_hist else (u, flags)

    def density(self, psi, weights=None):
        """rho_j = sum_b w_b |psi_b(r_j)|^2 on the FFT grid (C order [j1][j2][j3]); the
        Hellmann-Feynman derivative of sum_b w_b eps_b with respect to V_j is rho_j / (N1 N2 N3)."""
        psi = _cc(psi)
        nb = psi.shape[0]
        rho = np.zeros(self.grid)
        w = None if weights is None else _cd(np.broadcast_to(np.asarray(weights, np.float64), (nb,)))
        self._lib.orc_density(self._h, nb, _v(psi), None if w is None else _d(w), _d(rho))
        return rho

    def projector_gradient(self, psi, weights=None):
        """Derivatives of sum_b w_b <psi_b|V_NL|psi_b> with respect to the KB energies d_p
        (shape nproj) and the projector centres R_p (shape nproj x 3)."""
        psi = _cc(psi)
        nb = psi.shape[0]
        dd = np.zeros(self.nproj)
        dR = np.zeros((self.nproj, 3))
        w = None if weights is None else _cd(np.broadcast_to(np.asarray(weights, np.float64), (nb,)))
        if self.nproj:
            self._lib.orc_projector_gradient(self._h, nb, _v(psi), None if w is None else _d(w), _d(dd), _d(dR))
        return dd, dR

    def paro(self, trial, n_outer, ncg, sigma_lb, variant=0, shift_mode=0):
        """ParO (variant 0), MParO I (variant 1) or MParO II (variant 2) from a trial block.

        Returns dict(eps, psi, hpsi, eps_hist, res_hist, sigma_hist, flags)."""
        psi = _cc(trial).copy()
        nb, ng = psi.shape
        hpsi = np.zeros_like(psi)
        eps = np.zeros(nb)
        eh = np.zeros((n_outer + 1, nb))
        rh = np.zeros((n_outer + 1, nb))
        sh = np.zeros(max(n_outer, 1))
        f = self._lib.orc_paro(self._h, nb, _v(psi), _v(hpsi), _d(eps), n_outer, ncg, int(variant),
                               int(shift_mode), float(sigma_lb), _d(eh), _d(rh), _d(sh))
        return dict(eps=eps, psi=psi, hpsi=hpsi, eps_hist=eh, res_hist=rh,
                    sigma_hist=sh[:n_outer], flags=int(f))
