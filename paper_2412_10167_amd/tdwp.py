"""ctypes binding of libtdwp.so (argument marshalling only; every step of the
propagation and analysis runs in the library's HIP kernels).

The library owns its device memory; PyTorch, when present, only supplies the
current HIP stream so that the library's work is ordered with the caller's.
"""
import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
PRECISIONS = {"fp64": 0, "fp32": 1, "bf16x3": 2, "fp16x3": 3}
EXPORTED_SYMBOLS = (
    "tdwp_plan", "tdwp_grid", "tdwp_diatomic_states", "tdwp_set_potential",
    "tdwp_spectral_bounds", "tdwp_set_initial_packet", "tdwp_propagate", "tdwp_step_index",
    "tdwp_get_packet", "tdwp_state_to_state", "tdwp_time_kernels", "tdwp_destroy",
    "tdwp_strerror", "tdwp_mlp_n_params", "tdwp_set_potential_mlp", "tdwp_mlp_params",
    "tdwp_mlp_gradient", "tdwp_mlp_eval", "tdwp_mlp_eval_noalloc", "tdwp_mlp_grid", "tdwp_autotune",
    "tdwp_set_option", "tdwp_get_stat", "tdwp_jshift", "tdwp_jshift_interpolate",
    "tdwp_cumulative_probability", "tdwp_cross_section", "tdwp_fit_jshift_b",
    "tdwp_set_packet_values", "tdwp_autocorrelation", "tdwp_energy_content",
    "tdwp_photo_cross_section", "tdwp_apply_hamiltonian", "tdwp_lowest_state",
    "tdwp_photo_packet", "tdwp_product_grid", "tdwp_product_diatomic_states",
    "tdwp_state_to_state_products",
)
OPTIONS = {"graphs": 0, "ang_tile": 1, "radial_grid": 2, "ang_kernel": 3, "fuse_r": 4,
           "ang_xcd": 5, "plane_r": 6}
STATS = {"graph_steps": 0, "ang_tile": 1, "matrix_core_path": 2, "ang_kernel": 3, "fuse_r": 4,
         "ring_len": 5, "plane_r": 6, "potential_bytes": 7}


class TdwpError(RuntimeError):
    def __init__(self, code, what):
        self.code = code
        super().__init__(f"{what}: {_strerror(code)} ({code})")


class Unit(ctypes.Structure):
    _fields_ = [("J", ctypes.c_int), ("parity", ctypes.c_int), ("omega_max", ctypes.c_int),
                ("n_packets", ctypes.c_int)]


class Config(ctypes.Structure):
    _fields_ = [
        ("n_r", ctypes.c_int), ("n_R", ctypes.c_int), ("n_gamma", ctypes.c_int),
        ("r_min", ctypes.c_double), ("r_max", ctypes.c_double),
        ("R_min", ctypes.c_double), ("R_max", ctypes.c_double),
        ("mass_A", ctypes.c_double), ("mass_B", ctypes.c_double), ("mass_C", ctypes.c_double),
        ("n_elec", ctypes.c_int),
        ("rad_cut", ctypes.c_double), ("rot_cut", ctypes.c_double),
        ("abs_r_start", ctypes.c_double), ("abs_r_strength", ctypes.c_double), ("abs_r_power", ctypes.c_int),
        ("abs_R_start", ctypes.c_double), ("abs_R_strength", ctypes.c_double), ("abs_R_power", ctypes.c_int),
        ("e_min", ctypes.c_double), ("e_max", ctypes.c_double),
        ("r_flux", ctypes.c_double), ("R_inf", ctypes.c_double),
        ("n_energy", ctypes.c_int), ("ecol_min", ctypes.c_double), ("ecol_max", ctypes.c_double),
        ("n_units", ctypes.c_int), ("units", ctypes.POINTER(Unit)),
        ("precision", ctypes.c_int),
        ("stream", ctypes.c_void_p),
        ("prod_arrangement", ctypes.c_int),
        ("prod_n_r", ctypes.c_int), ("prod_n_gamma", ctypes.c_int),
        ("prod_R_inf", ctypes.c_double), ("prod_r_min", ctypes.c_double),
        ("prod_r_max", ctypes.c_double),
    ]


class Packet(ctypes.Structure):
    _fields_ = [("unit", ctypes.c_int), ("slot", ctypes.c_int), ("v0", ctypes.c_int),
                ("j0", ctypes.c_int), ("omega0", ctypes.c_int), ("elec0", ctypes.c_int),
                ("E_v0j0", ctypes.c_double), ("R0", ctypes.c_double), ("width", ctypes.c_double),
                ("ecol_mean", ctypes.c_double), ("k_min_elastic", ctypes.c_long)]


class MlpOptions(ctypes.Structure):
    _fields_ = [("n_samples", ctypes.c_int), ("sample_idx", ctypes.POINTER(ctypes.c_long)),
                ("init_params", ctypes.POINTER(ctypes.c_float)), ("order", ctypes.POINTER(ctypes.c_int)),
                ("batch", ctypes.c_int), ("epochs", ctypes.c_int), ("lr", ctypes.c_double),
                ("lr_final", ctypes.c_double)]


class Channel(ctypes.Structure):
    _fields_ = [("elec", ctypes.c_int), ("v", ctypes.c_int), ("j", ctypes.c_int),
                ("omega", ctypes.c_int), ("energy", ctypes.c_double)]


_LIB = None


def library_path():
    return os.environ.get("TDWP_LIBRARY", os.path.join(HERE, "libtdwp.so"))


def load_library():
    """Loads the HIP library; raises if it has not been built (there is no fallback)."""
    global _LIB
    if _LIB is not None:
        return _LIB
    path = library_path()
    if not os.path.exists(path):
        raise RuntimeError(f"tdwp HIP library not found at {path}; build it with "
                           "`python -m paper_2412_10167_amd.build_lib` or __graft_entry__.build()")
    # torch ships its own copy of the HIP runtime and loads it by path; were the
    # library loaded first, the process would hold two runtimes and torch's streams
    # and device memory would be foreign to the library's.  Importing torch first
    # makes the library bind to that same runtime (both carry one soname).
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = ctypes.CDLL(path)
    dp = ctypes.POINTER(ctypes.c_double)
    P = ctypes.c_void_p
    lib.tdwp_plan.argtypes = [ctypes.POINTER(Config), ctypes.POINTER(ctypes.c_void_p)]
    lib.tdwp_grid.argtypes = [P, dp, dp, dp, dp]
    lib.tdwp_diatomic_states.argtypes = [P, dp, ctypes.c_int, ctypes.c_int, dp, dp]
    lib.tdwp_set_potential.argtypes = [P, ctypes.c_int, dp, ctypes.c_size_t]
    lib.tdwp_spectral_bounds.argtypes = [P, dp, dp]
    lib.tdwp_set_initial_packet.argtypes = [P, ctypes.POINTER(Packet), dp]
    lib.tdwp_propagate.argtypes = [P, ctypes.c_long, dp]
    lib.tdwp_step_index.argtypes = [P, ctypes.POINTER(ctypes.c_long)]
    lib.tdwp_get_packet.argtypes = [P, ctypes.c_int, ctypes.c_int, ctypes.c_int, dp]
    lib.tdwp_state_to_state.argtypes = [P, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                        ctypes.POINTER(Channel), dp, dp, dp]
    lib.tdwp_time_kernels.argtypes = [P, ctypes.c_long, ctypes.c_int, dp, ctypes.c_char_p,
                                      ctypes.c_size_t]
    fp = ctypes.POINTER(ctypes.c_float)
    lib.tdwp_mlp_n_params.argtypes = [P]
    lib.tdwp_set_potential_mlp.argtypes = [P, dp, ctypes.c_size_t, ctypes.POINTER(MlpOptions), dp]
    lib.tdwp_mlp_params.argtypes = [P, fp]
    lib.tdwp_mlp_gradient.argtypes = [P, fp, ctypes.c_int, dp, dp, dp, fp]
    lib.tdwp_mlp_eval.argtypes = [P, ctypes.c_int, dp, dp]
    lib.tdwp_mlp_eval_noalloc.argtypes = [P, ctypes.c_int, dp, dp]
    lib.tdwp_mlp_grid.argtypes = [P, dp]
    lib.tdwp_autotune.argtypes = [P, ctypes.c_int, ctypes.c_char_p, ctypes.c_size_t]
    lib.tdwp_set_option.argtypes = [P, ctypes.c_int, ctypes.c_long]
    lib.tdwp_get_stat.argtypes = [P, ctypes.c_int, ctypes.POINTER(ctypes.c_long)]
    lib.tdwp_destroy.argtypes = [P]
    ip = ctypes.POINTER(ctypes.c_int)
    ci, cd = ctypes.c_int, ctypes.c_double
    lib.tdwp_jshift.argtypes = [dp, dp, ci, ci, cd, ci, dp]
    lib.tdwp_jshift_interpolate.argtypes = [dp, dp, dp, ci, ci, ci, cd, ci, dp]
    lib.tdwp_cumulative_probability.argtypes = [ip, dp, ci, dp, ci, ip, ci, dp, ci, ci, dp]
    lib.tdwp_cross_section.argtypes = [dp, ci, dp, ci, cd, ci, dp]
    lib.tdwp_fit_jshift_b.argtypes = [dp, dp, dp, ci, ci, ci, cd, dp]
    cl = ctypes.c_long
    lib.tdwp_set_packet_values.argtypes = [P, ci, ci, dp]
    lib.tdwp_photo_packet.argtypes = [P, ci, ci, ci, ci, ci, ci, ci, ci, dp, dp, ci]
    lib.tdwp_product_grid.argtypes = [P, dp, dp, dp]
    lib.tdwp_product_diatomic_states.argtypes = [P, dp, ci, ci, dp, dp]
    lib.tdwp_state_to_state_products.argtypes = [P, ci, ci, ci, ctypes.POINTER(Channel), dp, dp]
    lib.tdwp_autocorrelation.argtypes = [P, ci, ci, cl, dp]
    lib.tdwp_apply_hamiltonian.argtypes = [P, ci, ci, dp, dp]
    lib.tdwp_lowest_state.argtypes = [P, ci, ci, dp, ci, dp, dp, dp]
    lib.tdwp_energy_content.argtypes = [dp, cl, cd, cd, dp, ci, dp]
    lib.tdwp_photo_cross_section.argtypes = [dp, cl, cd, cd, cd, dp, ci, dp]
    lib.tdwp_destroy.restype = None
    lib.tdwp_strerror.argtypes = [ctypes.c_int]
    lib.tdwp_strerror.restype = ctypes.c_char_p
    for name in EXPORTED_SYMBOLS:
        if name not in ("tdwp_destroy", "tdwp_strerror"):
            getattr(lib, name).restype = ctypes.c_int
    _LIB = lib
    return lib


def _strerror(code):
    try:
        return load_library().tdwp_strerror(code).decode()
    except Exception:  # library not loadable: plain code
        return "error"


def _ptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _f64(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def _check(code, what):
    if code < 0:
        raise TdwpError(code, what)
    return code


def _current_stream():
    try:
        import torch
        if torch.cuda.is_available():
            return torch.cuda.current_stream().cuda_stream
    except Exception:
        pass
    return None


class Plan:
    """One tdwp plan: a batch of partial waves on one grid, owned device memory."""

    def __init__(self, spec, precision="fp64", bounds=None, stream="current"):
        self.lib = load_library()
        self.spec = spec
        units = spec["units"]
        self._units = (Unit * len(units))(*[Unit(u["J"], u["parity"], u["omega_max"], u["n_packets"])
                                           for u in units])
        if stream == "current":
            stream = _current_stream()
        e_min, e_max = bounds if bounds is not None else (0.0, 0.0)
        c = Config(
            n_r=spec["n_r"], n_R=spec["n_R"], n_gamma=spec["n_gamma"],
            r_min=spec["r_min"], r_max=spec["r_max"], R_min=spec["R_min"], R_max=spec["R_max"],
            mass_A=spec["mass_A"], mass_B=spec["mass_B"], mass_C=spec["mass_C"],
            n_elec=spec["n_elec"], rad_cut=spec["rad_cut"], rot_cut=spec["rot_cut"],
            abs_r_start=spec["abs_r_start"], abs_r_strength=spec["abs_r_strength"],
            abs_r_power=spec["abs_r_power"],
            abs_R_start=spec["abs_R_start"], abs_R_strength=spec["abs_R_strength"],
            abs_R_power=spec["abs_R_power"],
            e_min=e_min, e_max=e_max, r_flux=spec["r_flux"], R_inf=spec["R_inf"],
            n_energy=spec["n_energy"], ecol_min=spec["ecol_min"], ecol_max=spec["ecol_max"],
            n_units=len(units), units=self._units, precision=PRECISIONS[precision],
            stream=stream)
        prod = spec.get("products")
        if prod:
            c.prod_arrangement = {"C": 1, "B": 2}[prod["arrangement"]]
            c.prod_n_r, c.prod_n_gamma = prod["n_r"], prod["n_gamma"]
            c.prod_R_inf, c.prod_r_min, c.prod_r_max = prod["R_inf"], prod["r_min"], prod["r_max"]
        self._cfg = c
        h = ctypes.c_void_p()
        _check(self.lib.tdwp_plan(ctypes.byref(c), ctypes.byref(h)), "tdwp_plan")
        self.handle = h

    # -- plan queries ------------------------------------------------------
    def grid(self):
        s = self.spec
        r, R = np.empty(s["n_r"]), np.empty(s["n_R"])
        x, w = np.empty(s["n_gamma"]), np.empty(s["n_gamma"])
        _check(self.lib.tdwp_grid(self.handle, _ptr(r), _ptr(R), _ptr(x), _ptr(w)), "tdwp_grid")
        return r, R, x, w

    def diatomic_states(self, v_asym, j, n_states):
        v = _f64(v_asym)
        e = np.empty(n_states)
        chi = np.empty((n_states, self.spec["n_r"]))
        _check(self.lib.tdwp_diatomic_states(self.handle, _ptr(v), j, n_states, _ptr(e), _ptr(chi)),
               "tdwp_diatomic_states")
        return e, chi

    def set_potential(self, vtable, mode=0):
        v = _f64(vtable)
        _check(self.lib.tdwp_set_potential(self.handle, mode, _ptr(v), v.size), "tdwp_set_potential")

    def spectral_bounds(self):
        a, b = ctypes.c_double(), ctypes.c_double()
        _check(self.lib.tdwp_spectral_bounds(self.handle, ctypes.byref(a), ctypes.byref(b)),
               "tdwp_spectral_bounds")
        return a.value, b.value

    def set_initial_packet(self, packet, chi0, E_v0j0):
        p = Packet(unit=packet["unit"], slot=packet["slot"], v0=packet["v0"], j0=packet["j0"],
                   omega0=packet["omega0"], elec0=packet["elec0"], E_v0j0=E_v0j0,
                   R0=packet["R0"], width=packet["width"], ecol_mean=packet["ecol_mean"],
                   k_min_elastic=packet.get("k_min_elastic", 0))
        c = _f64(chi0)
        _check(self.lib.tdwp_set_initial_packet(self.handle, ctypes.byref(p), _ptr(c)),
               "tdwp_set_initial_packet")

    def n_packets(self):
        return sum(u["n_packets"] for u in self.spec["units"])

    def propagate(self, n_steps, norms=True):
        out = np.empty((self.n_packets(), n_steps)) if norms else None
        _check(self.lib.tdwp_propagate(self.handle, n_steps, _ptr(out) if norms else None),
               "tdwp_propagate")
        return out

    def step_index(self):
        k = ctypes.c_long()
        _check(self.lib.tdwp_step_index(self.handle, ctypes.byref(k)), "tdwp_step_index")
        return k.value

    def n_omega(self, unit):
        u = self.spec["units"][unit]
        lo = 0 if u["parity"] * (-1) ** u["J"] == 1 else 1
        return u["omega_max"] - lo + 1

    def get_packet(self, unit=0, slot=0, which=0):
        s = self.spec
        out = np.empty((self.n_omega(unit), s["n_elec"], s["n_gamma"], s["n_R"], s["n_r"]))
        _check(self.lib.tdwp_get_packet(self.handle, unit, slot, which, _ptr(out)), "tdwp_get_packet")
        return out

    def state_to_state(self, unit, slot, channels, reactive=True):
        """channels: list of dicts (elec, v, j, omega, energy, chi)."""
        s = self.spec
        n = len(channels)
        ch = (Channel * max(n, 1))(*[Channel(c["elec"], c["v"], c["j"], c["omega"], c["energy"])
                                     for c in channels])
        chi = _f64(np.array([c["chi"] for c in channels]) if n else np.zeros((1, s["n_r"])))
        p_inel = np.empty((n, s["n_energy"]))
        p_reac = np.empty((s["n_elec"], s["n_energy"]))
        _check(self.lib.tdwp_state_to_state(self.handle, unit, slot, n, ch, _ptr(chi),
                                            _ptr(p_inel) if n else None,
                                            _ptr(p_reac) if reactive else None),
               "tdwp_state_to_state")
        return p_inel, (p_reac if reactive else None)

    # -- learned potential ---------------------------------------------------
    def set_packet_values(self, unit, slot, u0):
        """Installs a photodissociation packet from values in the packet layout."""
        u = _f64(u0).ravel()
        n = self.n_omega(unit) * self.spec["n_elec"] * self.spec["n_gamma"] * self.spec["n_R"] \
            * self.spec["n_r"]
        if u.size != n:
            raise ValueError(f"packet of unit {unit} has {n} values, got {u.size}")
        _check(self.lib.tdwp_set_packet_values(self.handle, unit, slot, _ptr(u)),
               "tdwp_set_packet_values")

    def photo_packet(self, unit, slot, elec, J_i, M_i, p_i, om_lo_i, bound, dip, pol):
        """tdwp_photo_packet: bound [n_om_i][n_gamma][n_R][n_r], dip [3][n_gamma][n_R][n_r]
        (body-frame d_q, q = -1, 0, +1)."""
        b = _f64(bound)
        d = _f64(dip)
        s = self.spec
        pts = s["n_gamma"] * s["n_R"] * s["n_r"]
        if b.size % pts or d.size != 3 * pts:
            raise ValueError("bound / dip do not match the plan's grid")
        self._photo_keep = (b, d)
        _check(self.lib.tdwp_photo_packet(self.handle, unit, slot, elec, J_i, M_i, p_i, om_lo_i,
                                          b.size // pts, _ptr(b), _ptr(d), pol), "tdwp_photo_packet")

    def product_grid(self):
        pr = self.spec["products"]
        r = np.empty(pr["n_r"])
        x = np.empty(pr["n_gamma"])
        w = np.empty(pr["n_gamma"])
        _check(self.lib.tdwp_product_grid(self.handle, _ptr(r), _ptr(x), _ptr(w)), "tdwp_product_grid")
        return r, x, w

    def product_diatomic_states(self, v_asym, j, n_states):
        n = self.spec["products"]["n_r"]
        e = np.empty(n_states)
        chi = np.empty((n_states, n))
        _check(self.lib.tdwp_product_diatomic_states(self.handle, _ptr(_f64(v_asym)), j, n_states,
                                                     _ptr(e), _ptr(chi)), "tdwp_product_diatomic_states")
        return e, chi

    def state_to_state_products(self, unit, slot, channels):
        """|S'|^2 [n_ch][n_energy] of product channels (dicts elec, v, j, energy, chi)."""
        nE = self.spec["n_energy"]
        n = self.spec["products"]["n_r"]
        n_ch = len(channels)
        arr = (Channel * max(n_ch, 1))(*[Channel(c["elec"], c["v"], c["j"], c.get("omega", 0),
                                                 c["energy"]) for c in channels])
        chi = np.ascontiguousarray(np.array([c["chi"] for c in channels], dtype=np.float64)
                                   .reshape(n_ch, n))
        out = np.empty((n_ch, nE))
        _check(self.lib.tdwp_state_to_state_products(self.handle, unit, slot, n_ch, arr,
                                                     _ptr(chi), _ptr(out)),
               "tdwp_state_to_state_products")
        return out

    def apply_hamiltonian(self, u, unit=0, slot=0):
        """H u (undamped) for a vector in the layout of packet (unit, slot); no packet
        may be installed."""
        x = _f64(u).ravel()
        n = self.n_omega(unit) * self.spec["n_elec"] * self.spec["n_gamma"] * self.spec["n_R"] \
            * self.spec["n_r"]
        if x.size != n:
            raise ValueError(f"packet of unit {unit} has {n} values, got {x.size}")
        out = np.empty_like(x)
        _check(self.lib.tdwp_apply_hamiltonian(self.handle, unit, slot, _ptr(x), _ptr(out)),
               "tdwp_apply_hamiltonian")
        return out.reshape(np.shape(u))

    def lowest_state(self, guess, n_iter=300, unit=0, slot=0):
        """(energy, psi, residual) of the lowest eigenstate of H in the space of packet
        (unit, slot), by the library's Lanczos iteration from `guess`."""
        g = _f64(guess).ravel()
        psi = np.empty_like(g)
        e, r = ctypes.c_double(), ctypes.c_double()
        _check(self.lib.tdwp_lowest_state(self.handle, unit, slot, _ptr(g), n_iter,
                                          ctypes.byref(e), _ptr(psi), ctypes.byref(r)),
               "tdwp_lowest_state")
        return e.value, psi.reshape(np.shape(guess)), r.value

    def autocorrelation(self, unit=0, slot=0, n=None):
        """C_0 .. C_{n-1} = <u_0|u_k> of a photodissociation packet (default: up to the
        current step)."""
        if n is None:
            n = self.step_index() + 1
        out = np.empty(n)
        _check(self.lib.tdwp_autocorrelation(self.handle, unit, slot, n, _ptr(out)),
               "tdwp_autocorrelation")
        return out

    def mlp_n_params(self):
        return _check(self.lib.tdwp_mlp_n_params(self.handle), "tdwp_mlp_n_params")

    def set_potential_mlp(self, vtable, sample_idx, init_params, order, batch=1024, epochs=10,
                          lr=1e-3, lr_final=0.0):
        """Trains the surrogate on the device; returns (final loss, rms error, max error)."""
        v = _f64(vtable)
        idx = np.ascontiguousarray(sample_idx, dtype=np.int64)
        th = np.ascontiguousarray(init_params, dtype=np.float32)
        od = np.ascontiguousarray(order, dtype=np.int32)
        self._mlp_keep = (idx, th, od)
        o = MlpOptions(n_samples=idx.size,
                       sample_idx=idx.ctypes.data_as(ctypes.POINTER(ctypes.c_long)),
                       init_params=th.ctypes.data_as(ctypes.POINTER(ctypes.c_float)),
                       order=od.ctypes.data_as(ctypes.POINTER(ctypes.c_int)),
                       batch=batch, epochs=epochs, lr=lr, lr_final=lr_final)
        rep = np.zeros(3)
        _check(self.lib.tdwp_set_potential_mlp(self.handle, _ptr(v), v.size, ctypes.byref(o), _ptr(rep)),
               "tdwp_set_potential_mlp")
        return tuple(rep)

    def mlp_params(self):
        out = np.empty(self.mlp_n_params(), dtype=np.float32)
        _check(self.lib.tdwp_mlp_params(self.handle, out.ctypes.data_as(ctypes.POINTER(ctypes.c_float))),
               "tdwp_mlp_params")
        return out

    def mlp_gradient(self, params, dist, v):
        th = np.ascontiguousarray(params, dtype=np.float32)
        d = _f64(dist)
        vv = _f64(v)
        g = np.empty(th.size, dtype=np.float32)
        loss = ctypes.c_double()
        _check(self.lib.tdwp_mlp_gradient(self.handle, th.ctypes.data_as(ctypes.POINTER(ctypes.c_float)),
                                          d.shape[0], _ptr(d), _ptr(vv), ctypes.byref(loss),
                                          g.ctypes.data_as(ctypes.POINTER(ctypes.c_float))),
               "tdwp_mlp_gradient")
        return loss.value, g

    def mlp_eval(self, dist):
        d = _f64(dist)
        out = np.empty((d.shape[0], self.spec["n_elec"] * (self.spec["n_elec"] + 1) // 2))
        _check(self.lib.tdwp_mlp_eval(self.handle, d.shape[0], _ptr(d), _ptr(out)), "tdwp_mlp_eval")
        return out

    def mlp_eval_noalloc(self, dist):
        """tdwp_mlp_eval_noalloc: the same inference staged in the library's fixed
        device scratch (no device allocation)."""
        d = _f64(dist)
        out = np.empty((d.shape[0], self.spec["n_elec"] * (self.spec["n_elec"] + 1) // 2))
        _check(self.lib.tdwp_mlp_eval_noalloc(self.handle, d.shape[0], _ptr(d), _ptr(out)),
               "tdwp_mlp_eval_noalloc")
        return out

    def set_option(self, name, value):
        _check(self.lib.tdwp_set_option(self.handle, OPTIONS[name], int(value)), "tdwp_set_option")

    def stat(self, name):
        v = ctypes.c_long()
        _check(self.lib.tdwp_get_stat(self.handle, STATS[name], ctypes.byref(v)), "tdwp_get_stat")
        return v.value

    def autotune(self, steps=5):
        """Times the tile variants of the step kernels and keeps the fastest (call
        before setting packets).  Returns the report text."""
        buf = ctypes.create_string_buffer(4096)
        _check(self.lib.tdwp_autotune(self.handle, steps, buf, 4096), "tdwp_autotune")
        return buf.value.decode()

    def mlp_grid(self):
        s = self.spec
        npair = s["n_elec"] * (s["n_elec"] + 1) // 2
        out = np.empty((npair, s["n_gamma"], s["n_R"], s["n_r"]))
        _check(self.lib.tdwp_mlp_grid(self.handle, _ptr(out)), "tdwp_mlp_grid")
        return out

    def time_kernels(self, n_steps, n_max=8):
        avg = np.zeros(n_max)
        names = ctypes.create_string_buffer(512)
        n = _check(self.lib.tdwp_time_kernels(self.handle, n_steps, n_max, _ptr(avg), names, 512),
                   "tdwp_time_kernels")
        keys = names.value.decode().split(";")[:n]
        return dict(zip(keys, avg[:n]))

    def close(self):
        if getattr(self, "handle", None):
            self.lib.tdwp_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


# ---- partial-wave sums (host functions of the library; no plan, no device) ----

def _i32(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.int32))


def _iptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int))


def jshift(p_ref, energies, J_ref, B, J):
    """p_ref J-shifted from J_ref to J (tdwp_jshift)."""
    p, e = _f64(p_ref), _f64(energies)
    out = np.empty_like(e)
    _check(load_library().tdwp_jshift(_ptr(p), _ptr(e), e.size, J_ref, B, J, _ptr(out)),
           "tdwp_jshift")
    return out


def jshift_interpolate(p1, p2, energies, J1, J2, B, J):
    """Probability at J from the computed J1 and J2 curves (tdwp_jshift_interpolate)."""
    a, b, e = _f64(p1), _f64(p2), _f64(energies)
    out = np.empty_like(e)
    _check(load_library().tdwp_jshift_interpolate(_ptr(a), _ptr(b), _ptr(e), e.size, J1, J2, B, J,
                                                  _ptr(out)), "tdwp_jshift_interpolate")
    return out


def cumulative_probability(J_calc, B, p, energies, J_max, fam_jmin=None):
    """Cumulative probability c[n_f][n_e] from p[n_calc][n_fam][n_f][n_e]
    (tdwp_cumulative_probability)."""
    jc, bb, pp, e = _i32(J_calc), _f64(B), _f64(p), _f64(energies)
    if pp.ndim != 4 or pp.shape[0] != jc.size or pp.shape[3] != e.size or bb.size != jc.size:
        raise ValueError("p must be [n_calc][n_fam][n_f][n_e] with n_calc = len(J_calc) = len(B)")
    n_fam, n_f = pp.shape[1], pp.shape[2]
    jm = None
    if fam_jmin is not None:
        jm = _i32(fam_jmin)
        if jm.size != n_fam:
            raise ValueError("fam_jmin needs one entry per family")
    out = np.empty((n_f, e.size))
    _check(load_library().tdwp_cumulative_probability(
        _iptr(jc), _ptr(bb), jc.size, _ptr(pp), n_fam, None if jm is None else _iptr(jm), n_f,
        _ptr(e), e.size, J_max, _ptr(out)), "tdwp_cumulative_probability")
    return out


def cross_section(c, e_col, mu, j0):
    """Integral cross section [n_f][n_e] in bohr^2 from cumulative probabilities
    (tdwp_cross_section)."""
    cc, e = _f64(c), _f64(e_col)
    if cc.ndim == 1:
        cc = cc[None, :]
    if cc.shape[1] != e.size:
        raise ValueError("c must be [n_f][n_e]")
    out = np.empty_like(cc)
    _check(load_library().tdwp_cross_section(_ptr(cc), cc.shape[0], _ptr(e), e.size, mu, j0,
                                             _ptr(out)), "tdwp_cross_section")
    return out


def fit_jshift_b(p1, p2, energies, J1, J2, B_max):
    """Fitted rotational constant of the interval [J1, J2] (tdwp_fit_jshift_b)."""
    a, b, e = _f64(p1), _f64(p2), _f64(energies)
    out = ctypes.c_double()
    _check(load_library().tdwp_fit_jshift_b(_ptr(a), _ptr(b), _ptr(e), e.size, J1, J2, B_max,
                                            ctypes.byref(out)), "tdwp_fit_jshift_b")
    return out.value


# ---- photodissociation spectra (host functions of the library) ----

def energy_content(C, e_min, e_max, energies):
    """a_0(E) from an autocorrelation series (tdwp_energy_content)."""
    c, e = _f64(C), _f64(energies)
    out = np.empty_like(e)
    _check(load_library().tdwp_energy_content(_ptr(c), c.size, e_min, e_max, _ptr(e), e.size,
                                              _ptr(out)), "tdwp_energy_content")
    return out


def photo_cross_section(C, e_min, e_max, E_i, hnu):
    """sigma(h nu) in bohr^2 from an autocorrelation series (tdwp_photo_cross_section)."""
    c, h = _f64(C), _f64(hnu)
    out = np.empty_like(h)
    _check(load_library().tdwp_photo_cross_section(_ptr(c), c.size, e_min, e_max, E_i, _ptr(h),
                                                   h.size, _ptr(out)),
           "tdwp_photo_cross_section")
    return out
