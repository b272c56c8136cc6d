"""Thin Python binding over libparo (argument marshalling only).

PyTorch provides device memory and the stream; every numerical step runs in
the library's HIP kernels.  Orbital blocks are torch.complex128 tensors of
shape (bands, ld) on the GPU, one band per row (band-major), ld >= n_g.
"""
from __future__ import annotations

import ctypes as C

import numpy as np

from . import _lib as L


def _torch():
    import torch
    return torch


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else None


def _stream(device):
    torch = _torch()
    return C.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def sphere_enumerate(cell, ecut):
    """Miller indices (n_g x 3, int32, canonical order) of the cutoff sphere and n_max."""
    lib = L.load()
    cell = np.ascontiguousarray(cell, np.float64).reshape(9)
    ng = C.c_int64()
    nmax = np.zeros(3, np.int32)
    dp = cell.ctypes.data_as(C.POINTER(C.c_double))
    L.check(lib.paro_sphere_enumerate(dp, float(ecut), 0, None, C.byref(ng),
                                      nmax.ctypes.data_as(C.POINTER(C.c_int32))), "paro_sphere_enumerate")
    mil = np.zeros((ng.value, 3), np.int32)
    L.check(lib.paro_sphere_enumerate(dp, float(ecut), ng.value, mil.ctypes.data_as(C.POINTER(C.c_int32)),
                                      C.byref(ng), None), "paro_sphere_enumerate")
    return mil, nmax


def grid_size(nmax):
    lib = L.load()
    nm = np.ascontiguousarray(nmax, np.int32)
    out = np.zeros(3, np.int32)
    L.check(lib.paro_grid_size(nm.ctypes.data_as(C.POINTER(C.c_int32)), out.ctypes.data_as(C.POINTER(C.c_int32))),
            "paro_grid_size")
    return out


def _projectors(projs):
    arr = (L.Projector * max(1, len(projs)))()
    for i, p in enumerate(projs):
        arr[i].center[:] = [float(x) for x in p["center"]]
        arr[i].l, arr[i].m = int(p["l"]), int(p["m"])
        arr[i].width, arr[i].d = float(p["width"]), float(p["d"])
    return arr


class Plan:
    """A fixed Hamiltonian (cell, cutoff, local potential, KB projectors) on one GPU."""

    def __init__(self, cell, ecut, vloc, projectors=(), device="cuda:0", miller=None):
        torch = _torch()
        self.lib = L.load()
        self.device = torch.device(device)
        cell = np.ascontiguousarray(cell, np.float64).reshape(9)
        v = np.ascontiguousarray(vloc, np.float64)
        if miller is None:
            miller, _ = sphere_enumerate(cell, ecut)
        self.miller = np.ascontiguousarray(miller, np.int32)
        self._keep = (cell, v, self.miller, _projectors(projectors))
        prob = L.Problem()
        prob.cell[:] = list(cell)
        prob.ecut = float(ecut)
        prob.grid[:] = list(v.shape)
        prob.n_g = len(self.miller)
        prob.miller = self.miller.ctypes.data_as(C.POINTER(C.c_int32))
        prob.vloc = v.ctypes.data_as(C.POINTER(C.c_double))
        prob.n_proj = len(projectors)
        prob.proj = self._keep[3] if len(projectors) else None
        nbytes = C.c_size_t()
        L.check(self.lib.paro_plan_bytes(C.byref(prob), C.byref(nbytes)), "paro_plan_bytes")
        with torch.cuda.device(self.device):
            self.buf = torch.empty(nbytes.value + 256, dtype=torch.uint8, device=self.device)
            off = (-self.buf.data_ptr()) % 256
            h = C.c_void_p()
            L.check(self.lib.paro_plan_create(C.byref(prob), C.c_void_p(self.buf.data_ptr() + off), nbytes.value,
                                              _stream(self.device), C.byref(h)), "paro_plan_create")
        self.h = h
        info = L.PlanInfo()
        L.check(self.lib.paro_plan_get_info(self.h, C.byref(info)), "paro_plan_get_info")
        self.ng = int(info.n_g)
        self.nmax = tuple(info.nmax)
        self.grid = tuple(info.grid)
        self.n_sticks = int(info.n_sticks)
        self.n_proj = int(info.n_proj)
        self.omega = float(info.omega)
        self._ws = {}

    def __del__(self):
        h = getattr(self, "h", None)
        if h is not None and h.value:
            try:
                self.lib.paro_plan_destroy(h)
            except Exception:
                pass
            self.h = None

    # -------------------------------------------------------------- plumbing
    def _sync_stream(self):
        L.check(self.lib.paro_plan_set_stream(self.h, _stream(self.device)), "paro_plan_set_stream")

    def workspace_bytes(self, nb):
        n = C.c_size_t()
        L.check(self.lib.paro_workspace_bytes(self.h, int(nb), C.byref(n)), "paro_workspace_bytes")
        return n.value

    def workspace(self, nb):
        """A cached device workspace for calls on up to nb bands."""
        torch = _torch()
        nb = int(nb)
        ws = self._ws.get(nb)
        if ws is None:
            n = self.workspace_bytes(nb)
            raw = torch.empty(n + 256, dtype=torch.uint8, device=self.device)
            off = (-raw.data_ptr()) % 256
            ws = (raw, raw.data_ptr() + off, n)
            self._ws[nb] = ws
        return C.c_void_p(ws[1]), ws[2]

    def new_block(self, nb, ld=None):
        torch = _torch()
        ld = ld or self.ng
        return torch.zeros((nb, ld), dtype=torch.complex128, device=self.device)

    def _check_block(self, x, nb=None):
        torch = _torch()
        assert x.dtype == torch.complex128 and x.device == self.device and x.dim() == 2
        assert x.stride(1) == 1 and x.stride(0) >= self.ng, "band-major complex128 block with ld >= n_g"
        if nb is not None:
            assert x.shape[0] >= nb

    # -------------------------------------------------------------- tuning
    def set_schedule(self, precision, schedule, bands):
        """Line schedule and bands per work-group of the plane stage for one precision
        (paro_plan_set_schedule)."""
        self._sync_stream()
        L.check(self.lib.paro_plan_set_schedule(self.h, int(precision), int(schedule), int(bands)),
                "paro_plan_set_schedule")

    def get_schedule(self, precision):
        s, b, n = C.c_int32(), C.c_int32(), C.c_int32()
        L.check(self.lib.paro_plan_get_schedule(self.h, int(precision), C.byref(s), C.byref(b), C.byref(n)),
                "paro_plan_get_schedule")
        return dict(schedule=s.value, bands=b.value, n_schedules=n.value)

    def autotune(self, nb, force=False):
        """Time the plane stage's schedules and bands per work-group on nb bands and keep the
        fastest for both precisions (paro_plan_autotune)."""
        ws, n = self.workspace(nb)
        self._sync_stream()
        r = L.TuneResult()
        L.check(self.lib.paro_plan_autotune(self.h, int(nb), ws, n, L.TUNE_FORCE if force else 0, C.byref(r)),
                "paro_plan_autotune")
        return dict(schedule=list(r.schedule), bands=list(r.bands), ms=list(r.ms), ms_default=list(r.ms_default),
                    candidates=int(r.candidates), cached=bool(r.cached))

    # -------------------------------------------------------------- data
    def kinetic(self):
        torch = _torch()
        out = torch.empty(self.ng, dtype=torch.float64, device=self.device)
        self._sync_stream()
        L.check(self.lib.paro_get_kinetic(self.h, _ptr(out)), "paro_get_kinetic")
        return out

    def projectors(self):
        torch = _torch()
        out = torch.zeros((self.n_proj, self.ng), dtype=torch.complex128, device=self.device)
        self._sync_stream()
        L.check(self.lib.paro_get_projectors(self.h, _ptr(out)), "paro_get_projectors")
        return out

    # -------------------------------------------------------------- hot path
    def apply_h(self, psi, shift=None, out=None):
        """(H - shift_b) psi_b for every row b of psi."""
        self._check_block(psi)
        nb = psi.shape[0]
        out = out if out is not None else _torch().empty_like(psi)
        ws, n = self.workspace((nb + 1) // 2)
        self._sync_stream()
        L.check(self.lib.paro_apply_h(self.h, nb, _ptr(psi), psi.stride(0), _ptr(shift), _ptr(out), ws, n),
                "paro_apply_h")
        return out

    def apply_h_f32(self, psi, shift=None, out=None, bf16=False):
        """(H - shift_b) psi_b in single precision; psi: band-major complex64 block.  bf16:
        the projector products as split-BF16 products (paro_apply_h_f32_bf16)."""
        torch = _torch()
        assert psi.dtype == torch.complex64 and psi.device == self.device and psi.dim() == 2
        assert psi.stride(1) == 1 and psi.stride(0) >= self.ng
        nb = psi.shape[0]
        out = out if out is not None else torch.empty_like(psi)
        ws, n = self.workspace((nb + 1) // 2)
        self._sync_stream()
        name = "paro_apply_h_f32_bf16" if bf16 else "paro_apply_h_f32"
        L.check(getattr(self.lib, name)(self.h, nb, _ptr(psi), psi.stride(0), _ptr(shift), _ptr(out), ws, n), name)
        return out

    def density(self, psi, weights=None, out=None):
        """rho_j = sum_b w_b |psi_b(r_j)|^2 on the FFT grid (float64, shape grid, C order).
        For eigenpairs, d(sum_b w_b eps_b)/d vloc_j = rho_j / (N1 N2 N3)."""
        torch = _torch()
        self._check_block(psi)
        nb = psi.shape[0]
        if weights is not None:
            assert weights.dtype == torch.float64 and weights.device == self.device and weights.numel() >= nb
            weights = weights.contiguous()
        out = out if out is not None else torch.empty(self.grid, dtype=torch.float64, device=self.device)
        assert out.dtype == torch.float64 and out.is_contiguous() and tuple(out.shape) == self.grid
        ws, n = self._aux_workspace("density", nb, self.lib.paro_density_workspace_bytes)
        self._sync_stream()
        L.check(self.lib.paro_density(self.h, nb, _ptr(psi), psi.stride(0), _ptr(weights), _ptr(out), ws, n),
                "paro_density")
        return out

    def projector_gradient(self, psi, weights=None):
        """Derivatives of sum_b w_b <psi_b|V_NL|psi_b> with respect to the KB energies (n_proj)
        and the projector centres (n_proj x 3); for eigenpairs, of sum_b w_b eps_b."""
        torch = _torch()
        self._check_block(psi)
        nb = psi.shape[0]
        if weights is not None:
            assert weights.dtype == torch.float64 and weights.device == self.device and weights.numel() >= nb
            weights = weights.contiguous()
        dd = torch.zeros(self.n_proj, dtype=torch.float64, device=self.device)
        dR = torch.zeros((self.n_proj, 3), dtype=torch.float64, device=self.device)
        ws, n = self._aux_workspace("projgrad", nb, self.lib.paro_projector_gradient_workspace_bytes)
        self._sync_stream()
        L.check(self.lib.paro_projector_gradient(self.h, nb, _ptr(psi), psi.stride(0), _ptr(weights), _ptr(dd),
                                                 _ptr(dR), ws, n), "paro_projector_gradient")
        return dd, dR

    def _aux_workspace(self, kind, nb, query):
        """A cached 256-byte aligned device workspace sized by query(plan, nb)."""
        torch = _torch()
        key = (kind, int(nb))
        ws = self._ws.get(key)
        if ws is None:
            n = C.c_size_t()
            L.check(query(self.h, int(nb), C.byref(n)), kind + " workspace query")
            raw = torch.empty(n.value + 256, dtype=torch.uint8, device=self.device)
            off = (-raw.data_ptr()) % 256
            ws = (raw, raw.data_ptr() + off, n.value)
            self._ws[key] = ws
        return C.c_void_p(ws[1]), ws[2]

    def source_solve_mixed(self, psi, hpsi, eps, shift, n_cg, u=None):
        """As source_solve, with FP32 PCG vectors on the correction u - psi; returns (u, band_flags)."""
        torch = _torch()
        self._check_block(psi)
        nb = psi.shape[0]
        u = u if u is not None else torch.empty_like(psi)
        flags = torch.zeros(nb, dtype=torch.int32, device=self.device)
        ws, n = self.workspace(nb)
        self._sync_stream()
        L.check(self.lib.paro_source_solve_mixed(self.h, nb, _ptr(psi), _ptr(hpsi), psi.stride(0), _ptr(eps),
                                                 _ptr(shift), int(n_cg), _ptr(u), _ptr(flags), ws, n),
                "paro_source_solve_mixed")
        return u, flags

    def source_solve(self, psi, hpsi, eps, shift, n_cg, u=None):
        """u_b from n_cg PCG steps on (H - shift_b) u_b = (eps_b - shift_b) psi_b; returns (u, band_flags)."""
        torch = _torch()
        self._check_block(psi)
        nb = psi.shape[0]
        u = u if u is not None else torch.empty_like(psi)
        flags = torch.zeros(nb, dtype=torch.int32, device=self.device)
        ws, n = self.workspace(nb)
        self._sync_stream()
        L.check(self.lib.paro_source_solve(self.h, nb, _ptr(psi), _ptr(hpsi), psi.stride(0), _ptr(eps), _ptr(shift),
                                           int(n_cg), _ptr(u), _ptr(flags), ws, n), "paro_source_solve")
        return u, flags

    def rayleigh_ritz(self, U, W, n_keep):
        """Ritz pairs of H on span of the rows of U (W = H U); returns (eps, psi, hpsi)."""
        torch = _torch()
        self._check_block(U)
        m = U.shape[0]
        assert W.stride(0) == U.stride(0)
        eps = torch.empty(n_keep, dtype=torch.float64, device=self.device)
        psi = torch.zeros((n_keep, U.stride(0)), dtype=torch.complex128, device=self.device)
        hpsi = torch.zeros_like(psi)
        ws, n = self.workspace((m + 1) // 2)
        self._sync_stream()
        L.check(self.lib.paro_rayleigh_ritz(self.h, m, int(n_keep), _ptr(U), _ptr(W), U.stride(0), _ptr(eps),
                                            _ptr(psi), _ptr(hpsi), ws, n), "paro_rayleigh_ritz")
        return eps, psi, hpsi

    def residual_norms(self, psi, hpsi, eps):
        torch = _torch()
        nb = psi.shape[0]
        res = torch.empty(nb, dtype=torch.float64, device=self.device)
        ws, n = self.workspace(nb)
        self._sync_stream()
        L.check(self.lib.paro_residual_norms(self.h, nb, _ptr(psi), _ptr(hpsi), psi.stride(0), _ptr(eps), _ptr(res),
                                             ws, n), "paro_residual_norms")
        return res

    def shift_lower_bound(self):
        """sigma_lb = min V + min(0, lambda_min(V_NL)) - 0.1, computed on the device (returns a float)."""
        torch = _torch()
        out = torch.empty(1, dtype=torch.float64, device=self.device)
        ws, n = self.workspace(max(1, (self.n_proj + 1) // 2))
        self._sync_stream()
        L.check(self.lib.paro_shift_lower_bound(self.h, _ptr(out), ws, n), "paro_shift_lower_bound")
        return float(out.item())

    def iterate(self, psi, n_outer, n_cg, sigma_lb, hpsi=None, eps=None, variant=L.VARIANT_PARO,
                shift_mode=L.SHIFT_FIXED, initial_rr=True, n_conv=None, tol_res=0.0, stats=True,
                precision=L.PREC_FP64):
        """ParO / MParO I / MParO II outer iterations; psi is updated in place.  precision:
        PREC_FP64, PREC_MIXED (FP32 source problems, FP64 Rayleigh-Ritz), or PREC_MIXED_BF16
        (PREC_MIXED with split-BF16 projector products in the source problems).

        Returns dict(psi, hpsi, eps, sigma, stats (rows x (2 nb + 2)) or None, n_done)."""
        torch = _torch()
        self._check_block(psi)
        nb = psi.shape[0]
        hpsi = hpsi if hpsi is not None else torch.zeros_like(psi)
        eps = eps if eps is not None else torch.zeros(nb, dtype=torch.float64, device=self.device)
        sigma = torch.zeros(1, dtype=torch.float64, device=self.device)
        st = torch.full((n_outer + 1, 2 * nb + 2), float("nan"), dtype=torch.float64,
                        device=self.device) if stats else None
        o = L.IterOpts(n_outer=int(n_outer), n_cg=int(n_cg), n_conv=int(n_conv or nb), shift_mode=int(shift_mode),
                       variant=int(variant), initial_rr=1 if initial_rr else 0, sigma_lb=float(sigma_lb),
                       tol_res=float(tol_res), precision=int(precision))
        ws, n = self.workspace(nb)
        done = C.c_int32()
        self._sync_stream()
        L.check(self.lib.paro_iterate(self.h, nb, _ptr(psi), _ptr(hpsi), psi.stride(0), _ptr(eps), _ptr(sigma),
                                      C.byref(o), _ptr(st), ws, n, C.byref(done)), "paro_iterate")
        return dict(psi=psi, hpsi=hpsi, eps=eps, sigma=sigma, stats=st, n_done=int(done.value))

    def capture_iterations(self, psi, hpsi, eps, n_outer, n_cg, sigma_lb, variant=L.VARIANT_PARO,
                           precision=L.PREC_FP64):
        """Capture n_outer fixed-shift outer iterations on (psi, hpsi, eps), in place and starting
        from their current contents, into a torch CUDA graph; replaying it continues the
        iteration.  With the fixed shift and no tolerance the library makes no host decision,
        so the whole loop is device work.  Returns the torch.cuda.CUDAGraph."""
        torch = _torch()
        self._check_block(psi)
        self.workspace(psi.shape[0])  # allocate outside the capture
        g = torch.cuda.CUDAGraph()
        s = torch.cuda.Stream(device=self.device)
        s.wait_stream(torch.cuda.current_stream(self.device))
        with torch.cuda.graph(g, stream=s):
            self.iterate(psi, n_outer, n_cg, sigma_lb, hpsi=hpsi, eps=eps, variant=variant,
                         shift_mode=L.SHIFT_FIXED, initial_rr=False, tol_res=0.0, stats=False, precision=precision)
        torch.cuda.current_stream(self.device).wait_stream(s)
        return g

    def truncated_gradient(self, trial, n_outer, n_cg, sigma, weights=None):
        """Band energy E = sum_b w_b eps_b after the initial Rayleigh-Ritz of the trial block and
        n_outer fixed-shift ParO outer iterations (as iterate() computes them), and its derivatives
        dE/dvloc (grid-shaped) and dE/dR (n_proj x 3) through the truncated iterations.
        Returns (E, dvloc, dR)."""
        torch = _torch()
        self._check_block(trial)
        nb = trial.shape[0]
        w = torch.ones(nb, dtype=torch.float64, device=self.device) if weights is None else \
            torch.as_tensor(weights, dtype=torch.float64, device=self.device).contiguous()
        assert w.shape == (nb,)
        e = torch.empty(1, dtype=torch.float64, device=self.device)
        dv = torch.empty(self.grid, dtype=torch.float64, device=self.device)
        dr = torch.empty((max(self.n_proj, 1), 3), dtype=torch.float64, device=self.device)
        n = C.c_size_t()
        L.check(self.lib.paro_truncated_gradient_workspace_bytes(self.h, nb, int(n_outer), int(n_cg), C.byref(n)),
                "paro_truncated_gradient_workspace_bytes")
        raw = torch.empty(n.value + 256, dtype=torch.uint8, device=self.device)
        off = (-raw.data_ptr()) % 256
        self._sync_stream()
        L.check(self.lib.paro_truncated_gradient(self.h, nb, _ptr(trial), trial.stride(0), float(sigma), int(n_outer),
                                                 int(n_cg), _ptr(w), _ptr(e), _ptr(dv), _ptr(dr),
                                                 C.c_void_p(raw.data_ptr() + off), n.value), "paro_truncated_gradient")
        return float(e.item()), dv, dr[: self.n_proj]

    def status(self):
        """Read and clear the sticky device status bits (synchronises)."""
        f = C.c_int32()
        self._sync_stream()
        L.check(self.lib.paro_get_status(self.h, C.byref(f)), "paro_get_status")
        return int(f.value)


def iterate_batch(plans, psis, n_outer, n_cg, sigma_lbs, variant=L.VARIANT_PARO, shift_mode=L.SHIFT_FIXED,
                  initial_rr=True, n_conv=None, tol_res=0.0, precision=L.PREC_FP64, streams=None, stats=False,
                  hpsis=None, epss=None):
    """ParO outer iterations on many independent cells in one library call (paro_iterate_batch).

    plans[i] and psis[i] (its band-major complex128 block, updated in place) form cell i;
    sigma_lbs[i] its shift bound; n_conv and n_cg may be lists.  streams: torch streams (default
    priority) the cells are spread over round-robin (None: one per cell, at most 8); the
    cells' work is ordered after the current stream's and the current stream waits for all of
    them at the end.  hpsis / epss: each cell's H psi and eps to continue from (with
    initial_rr=False), updated in place.  Returns a list of dict(psi, hpsi, eps, sigma, stats,
    n_done)."""
    torch = _torch()
    n = len(plans)
    assert n == len(psis) == len(sigma_lbs) and n > 0
    dev = plans[0].device
    cur = torch.cuda.current_stream(dev)
    if streams is None:
        streams = [torch.cuda.Stream(device=dev) for _ in range(min(n, 8))]
    out, opts = [], (L.IterOpts * n)()
    ncv = n_conv if isinstance(n_conv, (list, tuple)) else [n_conv] * n
    ncgs = n_cg if isinstance(n_cg, (list, tuple)) else [n_cg] * n
    for i, (pl, psi) in enumerate(zip(plans, psis)):
        pl._check_block(psi)
        nb = psi.shape[0]
        out.append(dict(psi=psi, hpsi=hpsis[i] if hpsis is not None else torch.zeros_like(psi),
                        eps=epss[i] if epss is not None else torch.zeros(nb, dtype=torch.float64, device=dev),
                        sigma=torch.zeros(1, dtype=torch.float64, device=dev),
                        stats=torch.full((n_outer + 1, 2 * nb + 2), float("nan"), dtype=torch.float64, device=dev)
                        if stats else None))
        opts[i] = L.IterOpts(n_outer=int(n_outer), n_cg=int(ncgs[i]), n_conv=int(ncv[i] or nb),
                             shift_mode=int(shift_mode), variant=int(variant), initial_rr=1 if initial_rr else 0,
                             sigma_lb=float(sigma_lbs[i]), tol_res=float(tol_res), precision=int(precision))
    wss = [pl.workspace(psi.shape[0]) for pl, psi in zip(plans, psis)]
    vp = lambda xs: (C.c_void_p * n)(*[x.value if isinstance(x, C.c_void_p) else x for x in xs])  # noqa: E731
    hplans = (C.c_void_p * n)(*[pl.h.value for pl in plans])
    nbs = (C.c_int32 * n)(*[psi.shape[0] for psi in psis])
    lds = (C.c_int64 * n)(*[psi.stride(0) for psi in psis])
    ptr = lambda t: t.data_ptr() if t is not None else None  # noqa: E731
    done = (C.c_int32 * n)()
    ev = torch.cuda.Event()
    ev.record(cur)
    for k, pl in enumerate(plans):
        st = streams[k % len(streams)]
        st.wait_event(ev)
        L.check(pl.lib.paro_plan_set_stream(pl.h, C.c_void_p(st.cuda_stream)), "paro_plan_set_stream")
    lib = plans[0].lib
    L.check(lib.paro_iterate_batch(n, hplans, nbs, vp([ptr(psi) for psi in psis]),
                                   vp([ptr(o["hpsi"]) for o in out]), lds, vp([ptr(o["eps"]) for o in out]),
                                   vp([ptr(o["sigma"]) for o in out]), opts,
                                   vp([ptr(o["stats"]) for o in out]), vp([w[0] for w in wss]),
                                   (C.c_size_t * n)(*[w[1] for w in wss]), done), "paro_iterate_batch")
    for st in streams:
        e = torch.cuda.Event()
        e.record(st)
        cur.wait_event(e)
    # the tensors were used on the cell streams: keep the allocator from reusing them early
    for k, o in enumerate(out):
        st = streams[k % len(streams)]
        for t in (o["psi"], o["hpsi"], o["eps"], o["sigma"], o["stats"]):
            if t is not None:
                t.record_stream(st)
    for k, o in enumerate(out):
        o["n_done"] = int(done[k])
    return out


def capture_batch(plans, psis, hpsis, epss, n_outer, n_cg, sigma_lbs, variant=L.VARIANT_PARO,
                  precision=L.PREC_FP64):
    """Capture n_outer fixed-shift outer iterations of a batch of cells on (psis, hpsis, epss),
    in place and from their current contents, into a torch CUDA graph; replaying it continues
    the iterations.  With the fixed shift, no tolerance and all cells on the capturing stream
    the batch enqueues kernels only.  Workspaces are allocated before the capture.  Returns
    the torch.cuda.CUDAGraph."""
    torch = _torch()
    dev = plans[0].device
    for pl, psi in zip(plans, psis):
        pl.workspace(psi.shape[0])
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream(device=dev)
    s.wait_stream(torch.cuda.current_stream(dev))
    with torch.cuda.graph(g, stream=s):
        iterate_batch(plans, psis, n_outer, n_cg, sigma_lbs, variant=variant, shift_mode=L.SHIFT_FIXED,
                      initial_rr=False, tol_res=0.0, precision=precision, streams=[s], hpsis=hpsis,
                      epss=epss)
    torch.cuda.current_stream(dev).wait_stream(s)
    return g


def zgemm_hn(A, B, device=None):
    """C = A^H B for column-major complex A (K x M) and B (K x N) given as torch tensors of
    shape (M, K) and (N, K) (rows = columns of the matrices).  Returns C as (N, M) (rows = columns)."""
    torch = _torch()
    M, K = A.shape
    N = B.shape[0]
    C_ = torch.empty((N, M), dtype=torch.complex128, device=A.device)
    ws = torch.empty(max(M * N * 16 * 64, 1024), dtype=torch.uint8, device=A.device)
    lib = L.load()
    L.check(lib.paro_zgemm_hn(_stream(A.device), M, N, K, _ptr(A), A.stride(0), _ptr(B), B.stride(0), _ptr(C_), M,
                              _ptr(ws), ws.numel()), "paro_zgemm_hn")
    return C_


def zgemm_hn_noalloc(A, B):
    """zgemm_hn through paro_zgemm_hn_noalloc: the library's fixed device scratch instead of a
    workspace (only C is allocated here, by torch)."""
    torch = _torch()
    M, K = A.shape
    N = B.shape[0]
    C_ = torch.empty((N, M), dtype=torch.complex128, device=A.device)
    lib = L.load()
    L.check(lib.paro_zgemm_hn_noalloc(_stream(A.device), M, N, K, _ptr(A), A.stride(0), _ptr(B), B.stride(0),
                                      _ptr(C_), M), "paro_zgemm_hn_noalloc")
    return C_


def zgemm_nn(A, B, C_=None, accumulate=False):
    """C = A B (+ C): A column-major M x K given as (K, M) tensor, B as (N, K), C as (N, M)."""
    torch = _torch()
    K, M = A.shape
    N = B.shape[0]
    if C_ is None:
        C_ = torch.zeros((N, M), dtype=torch.complex128, device=A.device)
    lib = L.load()
    L.check(lib.paro_zgemm_nn(_stream(A.device), M, N, K, _ptr(A), A.stride(0), _ptr(B), B.stride(0), _ptr(C_),
                              C_.stride(0), 1 if accumulate else 0), "paro_zgemm_nn")
    return C_


def heev(A):
    """Eigenpairs of a Hermitian matrix on the device.  A: (m, m) torch complex128 (row-major,
    i.e. the column-major A^T = conj(A)); returns (w ascending, V with V[:, k] the k-th vector)."""
    torch = _torch()
    m = A.shape[0]
    Acm = A.transpose(0, 1).contiguous()  # column-major storage of A
    w = torch.empty(m, dtype=torch.float64, device=A.device)
    V = torch.empty((m, m), dtype=torch.complex128, device=A.device)
    lib = L.load()
    n = C.c_size_t()
    L.check(lib.paro_heev_workspace_bytes(m, C.byref(n)), "paro_heev_workspace_bytes")
    ws = torch.empty(n.value + 256, dtype=torch.uint8, device=A.device)
    off = (-ws.data_ptr()) % 256
    L.check(lib.paro_heev(_stream(A.device), m, _ptr(Acm), _ptr(w), _ptr(V), C.c_void_p(ws.data_ptr() + off),
                          n.value), "paro_heev")
    return w, V.transpose(0, 1)
