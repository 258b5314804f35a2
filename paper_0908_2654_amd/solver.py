"""Python front end of librh: a handle bound to one device and stream.

PyTorch provides device memory (the workspace and the fields) and the
stream; every step of the method runs in the library's HIP kernels.
"""
from __future__ import annotations

import ctypes

import torch

from . import _lib
from ._lib import RhAdvanceStats, RhAdvectStats, RhParams, RhStepStats, check, lib

_F64 = ctypes.c_double


def _ptr(t):
    if t is None:
        return None
    if not isinstance(t, torch.Tensor):
        raise TypeError("fields must be torch tensors")
    if t.device.type != "cuda":
        raise ValueError("fields must live on the HIP device")
    if t.dtype != torch.float64 or not t.is_contiguous():
        raise ValueError("fields must be contiguous float64")
    return ctypes.c_void_p(t.data_ptr())


def params_from_workload(w, **overrides) -> RhParams:
    """Map a workloads.Workload onto the C parameter struct (no arithmetic)."""
    p = _lib.default_params()
    p.nx, p.ny, p.nz = (int(d) for d in w.dims)
    for i, b in enumerate(w.bc):
        p.bc[i] = int(b)
    p.box_comoving_cm = float(w.box_comoving_cm)
    p.isothermal = int(bool(w.isothermal))
    p.T_iso_K = float(w.T_iso)
    p.spectrum = int(w.spectrum)
    p.T_bb_K = float(w.T_bb)
    p.hnu0_eV = float(w.hnu0_eV)
    p.sigma0_cm2 = float(w.sigma0)
    p.rates = int(w.rates)
    p.alphaB_const = float(w.alphaB_const)
    p.cooling_mask = int(w.cooling)
    p.cosmology = int(w.cosmology)
    p.hubble_h = float(w.hubble_h)
    p.Omega_m = float(w.Omega_m)
    p.Omega_L = float(w.Omega_L)
    p.theta = float(w.theta)
    p.newton_tol = float(w.newton_tol)
    p.precision = int(w.precision)
    p.mg_pre = int(w.mg_pre)
    p.mg_post = int(w.mg_post)
    for k, v in overrides.items():
        if k == "bc":
            for i, b in enumerate(v):
                p.bc[i] = int(b)
            continue
        if not hasattr(p, k):
            raise AttributeError(k)
        setattr(p, k, v)
    return p


def workspace_bytes(p: RhParams) -> int:
    n = lib.rh_workspace_bytes(ctypes.byref(p))
    if n == 0:
        check(_lib.RH_EINVAL)
    return int(n)


def cosmology_at(p: RhParams, t: float):
    a, H = _F64(), _F64()
    check(lib.rh_cosmology_at(ctypes.byref(p), float(t), ctypes.byref(a), ctypes.byref(H)))
    return a.value, H.value


def cosmic_time(p: RhParams, a: float) -> float:
    t = _F64()
    check(lib.rh_cosmic_time(ctypes.byref(p), float(a), ctypes.byref(t)))
    return t.value


def residual_noalloc(params: RhParams, t, dt, nH, src, Un, U, out, stream=None) -> float:
    """f(U) of the step from U^n through rh_residual_noalloc (no handle, no
    workspace: the library's static scratch; grids up to 64^3 cells).
    out = (fE, fe, fn) preallocated tensors (entries may be None); returns
    the RMS norm."""
    En, en, nn = Un
    E, e, n = U
    fE, fe, fn = out
    st = torch.cuda.current_stream() if stream is None else stream
    norm = _F64()
    s = lib.rh_residual_noalloc(ctypes.byref(params), ctypes.c_void_p(st.cuda_stream), float(t),
                                float(dt), _ptr(nH), _ptr(src), _ptr(En), _ptr(en), _ptr(nn),
                                _ptr(E), _ptr(e), _ptr(n), _ptr(fE), _ptr(fe), _ptr(fn),
                                ctypes.byref(norm))
    check(s)
    return norm.value


class Solver:
    """Owns a workspace tensor and a library handle on one device/stream."""

    def __init__(self, params: RhParams, device="cuda", stream=None):
        self.params = params
        self.device = torch.device(device)
        if self.device.type != "cuda":
            raise ValueError("the solver runs on a HIP device")
        # the library records the current device at setup and launches there
        torch.cuda.init()
        if self.device.index is not None:
            torch.cuda.set_device(self.device)
        else:
            self.device = torch.device("cuda", torch.cuda.current_device())
        self.ws_bytes = workspace_bytes(params)
        self.ws = torch.empty(self.ws_bytes, dtype=torch.uint8, device=self.device)
        self.stream = torch.cuda.current_stream(self.device) if stream is None else stream
        h = ctypes.c_void_p()
        st = lib.rh_setup(ctypes.byref(params), ctypes.c_void_p(self.ws.data_ptr()),
                          self.ws_bytes, ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h))
        check(st)
        self._h = h

    @property
    def dims(self):
        p = self.params
        return (p.nx, p.ny, p.nz)

    def close(self):
        if getattr(self, "_h", None):
            lib.rh_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_kernel_timing(self, enable: bool):
        check(lib.rh_set_kernel_timing(self._h, int(bool(enable))), self._h)

    def kernel_timing(self, reset=True) -> dict:
        """{class: (total ms, launches)} since the last reset."""
        n = len(_lib.KERNEL_CLASSES)
        ms = (_F64 * n)()
        cnt = (ctypes.c_int64 * n)()
        check(lib.rh_get_kernel_timing(self._h, ms, cnt, n, int(bool(reset))), self._h)
        return {k: (ms[i], cnt[i]) for i, k in enumerate(_lib.KERNEL_CLASSES)}

    def constants(self) -> dict:
        out = (_F64 * 8)()
        check(lib.rh_get_constants(self._h, out, 8), self._h)
        keys = ["sigma_E", "K_Gamma", "K_G", "eps_bar", "hnu0", "h", "levels", "coarse_cells"]
        return dict(zip(keys, list(out)))

    def initial_state(self, nH, x0, T0, E0, E, e, nHI):
        """Fill (E, e, nHI) in place: uniform E0, ionised fraction x0 and the gas
        energy of temperature T0 (e may be None for isothermal runs)."""
        s = lib.rh_initial_state(self._h, _ptr(nH), float(x0), float(T0), float(E0), _ptr(E),
                                 _ptr(e), _ptr(nHI))
        check(s, self._h)

    def source_field(self, photon_rate, src):
        """src = 4 pi eta from photons/s per cell (in place into src)."""
        check(lib.rh_source_field(self._h, _ptr(photon_rate), _ptr(src)), self._h)

    def step(self, t, dt, nH, src, E, e, nHI) -> dict:
        """One implicit step in place on (E, e, nHI); returns the step statistics."""
        st = RhStepStats()
        s = lib.rh_implicit_step(self._h, float(t), float(dt), _ptr(nH), _ptr(src), _ptr(E),
                                 _ptr(e), _ptr(nHI), ctypes.byref(st))
        check(s, self._h)
        return st.as_dict()

    def advance(self, t0, t_end, dt0, tau_tol, dt_max, nH, src, E, e, nHI) -> dict:
        """Adaptive steps from t0 to t_end in place on (E, e, nHI); returns the
        controller statistics plus t_reached.  Raises RhError if it stops early."""
        st = RhAdvanceStats()
        tr = _F64()
        s = lib.rh_advance(self._h, float(t0), float(t_end), float(dt0), float(tau_tol),
                           float(dt_max), _ptr(nH), _ptr(src), _ptr(E), _ptr(e), _ptr(nHI),
                           ctypes.byref(st), ctypes.byref(tr))
        check(s, self._h)
        d = st.as_dict()
        d["t_reached"] = tr.value
        return d

    def advect(self, t0, dt, v, nH, E, e, nHI, cfl=0.9) -> dict:
        """Advect (nH, E, e, nHI) in place over [t0, t0 + dt] with the cell-centred
        velocity v = (vx, vy, vz) (operator split, step (iv)); returns the
        substep statistics."""
        st = RhAdvectStats()
        s = lib.rh_advect(self._h, float(t0), float(dt), _ptr(v[0]), _ptr(v[1]), _ptr(v[2]),
                          float(cfl), _ptr(nH), _ptr(E), _ptr(e), _ptr(nHI), ctypes.byref(st))
        check(s, self._h)
        return st.as_dict()

    def split_step(self, t0, dt, v, nH, src, E, e, nHI, cfl=0.9) -> dict:
        """One operator-split step in place: advection over dt, then the
        implicit step from the advected fields (steps (iv) and (v))."""
        adv = self.advect(t0, dt, v, nH, E, e, nHI, cfl)
        st = self.step(t0, dt, nH, src, E, e, nHI)
        st["advect"] = adv
        return st

    def residual(self, t, dt, nH, src, Un, U, want_fields=True):
        """f(U) of the step from U^n: returns (fE, fe, fn, norm)."""
        En, en, nn = Un
        E, e, n = U
        fE = torch.empty_like(E) if want_fields else None
        fe = torch.empty_like(E) if (want_fields and not self.params.isothermal) else None
        fn = torch.empty_like(E) if want_fields else None
        norm = _F64()
        s = lib.rh_residual(self._h, float(t), float(dt), _ptr(nH), _ptr(src), _ptr(En), _ptr(en),
                            _ptr(nn), _ptr(E), _ptr(e), _ptr(n), _ptr(fE), _ptr(fe), _ptr(fn),
                            ctypes.byref(norm))
        check(s, self._h)
        return fE, fe, fn, norm.value

    def schur_operator(self, t, dt, nH, src, Un, U):
        """The Schur operator at U: (diag, (cf_x, cf_y, cf_z)) with
        (S x)_P = diag_P x_P - sum_d (cf_d,P x_{P+e_d} + cf_d,P-e_d x_{P-e_d})."""
        En, en, nn = Un
        E, e, n = U
        diag = torch.empty_like(E)
        cf = tuple(torch.empty_like(E) for _ in range(3))
        s = lib.rh_schur_operator(self._h, float(t), float(dt), _ptr(nH), _ptr(src), _ptr(En),
                                  _ptr(en), _ptr(nn), _ptr(E), _ptr(e), _ptr(n), _ptr(diag),
                                  *(_ptr(c) for c in cf))
        check(s, self._h)
        return diag, cf

    def schur_solve(self, t, dt, nH, src, Un, U, b, rel_tol=1e-12, max_it=100):
        """Solve S x = b with the Schur operator at U; returns (x, iters, rel_res)."""
        En, en, nn = Un
        E, e, n = U
        x = torch.empty_like(b)
        it = ctypes.c_int32()
        rr = _F64()
        s = lib.rh_schur_solve(self._h, float(t), float(dt), _ptr(nH), _ptr(src), _ptr(En),
                               _ptr(en), _ptr(nn), _ptr(E), _ptr(e), _ptr(n), _ptr(b), _ptr(x),
                               float(rel_tol), int(max_it), ctypes.byref(it), ctypes.byref(rr))
        check(s, self._h)
        return x, it.value, rr.value

    def adjoint_step(self, t, dt, nH, src, Un, U1, lam, g_src, g_nH) -> dict:
        """Adjoint of one step: lam = (lE, le, lnHI) in/out, gradients accumulated."""
        En, en, nn = Un
        E1, e1, n1 = U1
        lE, le, ln = lam
        st = RhStepStats()
        s = lib.rh_adjoint_step(self._h, float(t), float(dt), _ptr(nH), _ptr(src), _ptr(En),
                                _ptr(en), _ptr(nn), _ptr(E1), _ptr(e1), _ptr(n1), _ptr(lE),
                                _ptr(le), _ptr(ln), _ptr(g_src), _ptr(g_nH), ctypes.byref(st))
        check(s, self._h)
        return st.as_dict()


# ---------------------------------------------------------------------------
# hydrogen + helium chemistry with multigroup radiation
# ---------------------------------------------------------------------------
def multigroup_params(edges_eV, y_he=0.0, sigma_power=3.0) -> _lib.RhMultigroupParams:
    """The C struct for lower group edges edges_eV (first = the hydrogen
    threshold), helium abundance n_He / n_H and the cross-sections' power law."""
    if not 1 <= len(edges_eV) <= _lib.MAX_GROUPS:
        raise ValueError(f"1 to {_lib.MAX_GROUPS} groups")
    m = _lib.RhMultigroupParams()
    m.groups = len(edges_eV)
    for i, v in enumerate(edges_eV):
        m.edge_eV[i] = float(v)
    m.y_he = float(y_he)
    m.sigma_power = float(sigma_power)
    return m


def multigroup_constants(p: RhParams, mg) -> dict:
    """Group constants (host): frac [G], sigma_E, K_Gamma, K_G [3][G] (HI,
    HeI, HeII) and eps_bar."""
    G = mg.groups
    n = 10 * G + 1
    out = (_F64 * n)()
    _lib.check_multigroup(lib.rh_multigroup_constants(ctypes.byref(p), ctypes.byref(mg), out, n))
    v = list(out)
    rows = lambda o: [v[o + s * G: o + (s + 1) * G] for s in range(3)]  # noqa: E731
    return {"frac": v[:G], "sigma_E": rows(G), "K_Gamma": rows(4 * G), "K_G": rows(7 * G),
            "eps_bar": v[10 * G]}


class MultigroupSolver:
    """Handle of the multigroup step on one device/stream.  Fields: E [G, *dims],
    e [*dims], y [3, *dims] (n_HI, n_HeI, n_HeII), float64, contiguous."""

    def __init__(self, params: RhParams, mg, device="cuda", stream=None):
        self.params = params
        self.mg = mg
        self.G = mg.groups
        self.device = torch.device(device)
        if self.device.type != "cuda":
            raise ValueError("the solver runs on a HIP device")
        torch.cuda.init()
        if self.device.index is not None:
            torch.cuda.set_device(self.device)
        else:
            self.device = torch.device("cuda", torch.cuda.current_device())
        nb = lib.rh_multigroup_workspace_bytes(ctypes.byref(params), ctypes.byref(mg))
        if nb == 0:
            _lib.check_multigroup(_lib.RH_EINVAL)
        self.ws = torch.empty(nb, dtype=torch.uint8, device=self.device)
        self.stream = torch.cuda.current_stream(self.device) if stream is None else stream
        h = ctypes.c_void_p()
        st = lib.rh_multigroup_setup(ctypes.byref(params), ctypes.byref(mg),
                                     ctypes.c_void_p(self.ws.data_ptr()), nb,
                                     ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h))
        _lib.check_multigroup(st)
        self._h = h

    @property
    def dims(self):
        p = self.params
        return (p.nx, p.ny, p.nz)

    def close(self):
        if getattr(self, "_h", None):
            lib.rh_multigroup_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def empty_state(self):
        """Uninitialised (E, e, y) of the right shapes on the device."""
        o = dict(dtype=torch.float64, device=self.device)
        e = None if self.params.isothermal else torch.empty(self.dims, **o)
        return torch.empty((self.G,) + self.dims, **o), e, torch.zeros((3,) + self.dims, **o)

    def initial_state(self, nH, x0, T0, E0, E, e, y):
        s = lib.rh_multigroup_initial_state(self._h, _ptr(nH), float(x0), float(T0), float(E0),
                                            _ptr(E), _ptr(e), _ptr(y))
        _lib.check_multigroup(s, self._h)

    def step(self, t, dt, nH, src, E, e, y) -> dict:
        st = RhStepStats()
        s = lib.rh_multigroup_step(self._h, float(t), float(dt), _ptr(nH), _ptr(src), _ptr(E),
                                   _ptr(e), _ptr(y), ctypes.byref(st))
        _lib.check_multigroup(s, self._h)
        return st.as_dict()

    def set_kernel_timing(self, enable: bool):
        _lib.check_multigroup(lib.rh_multigroup_set_kernel_timing(self._h, int(bool(enable))),
                              self._h)

    def kernel_timing(self, reset=True) -> dict:
        """{class: (total ms, launches)} since the last reset, summed over the groups."""
        n = len(_lib.KERNEL_CLASSES)
        ms = (_F64 * n)()
        cnt = (ctypes.c_int64 * n)()
        _lib.check_multigroup(lib.rh_multigroup_get_kernel_timing(self._h, ms, cnt, n,
                                                                  int(bool(reset))), self._h)
        return {k: (ms[i], cnt[i]) for i, k in enumerate(_lib.KERNEL_CLASSES)}

    def residual(self, t, dt, nH, src, Un, U):
        """f(U) of the step from U^n = (E, e, y): returns (fE, fe, fy, norm)."""
        En, en, yn = Un
        E, e, y = U
        fE = torch.empty_like(E)
        fe = None if self.params.isothermal else torch.empty_like(e)
        fy = torch.zeros_like(y)
        norm = _F64()
        s = lib.rh_multigroup_residual(self._h, float(t), float(dt), _ptr(nH), _ptr(src),
                                       _ptr(En), _ptr(en), _ptr(yn), _ptr(E), _ptr(e), _ptr(y),
                                       _ptr(fE), _ptr(fe), _ptr(fy), ctypes.byref(norm))
        _lib.check_multigroup(s, self._h)
        return fE, fe, fy, norm.value
