"""Thin ctypes binding of libsalec (include/salec.h).

Argument marshalling only: every step of the grid update runs in the HIP
library. PyTorch supplies the device buffer (a uint8 tensor sized by
``salec_plan``) and the stream. There is no CPU fallback: constructing a
``Salec`` without the built library or without a HIP device raises.
"""
from __future__ import annotations

import ctypes as C
import os
import re

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsalec.so")
HEADER = os.path.join(HERE, "..", "include", "salec.h")

SALEC_FP64, SALEC_MIXED = 0, 1
ERRORS = {-1: "SALEC_E_INVALID", -2: "SALEC_E_BUFFER", -3: "SALEC_E_HIP", -4: "SALEC_E_NONFINITE",
          -5: "SALEC_E_NEG_MASS", -6: "SALEC_E_DT_FLOOR"}


class Grid(C.Structure):
    _fields_ = [("n_r", C.c_int32), ("n_z", C.c_int32), ("pml_r", C.c_int32), ("pml_b", C.c_int32),
                ("nmat", C.c_int32), ("top_closed", C.c_int32), ("precision", C.c_int32),
                ("closure", C.c_int32)] + \
               [(n, C.c_double) for n in ("dr", "dz", "cfl", "dt_grow", "dt_max", "dt_floor", "t_stop",
                                          "q_lin", "q_quad")] + \
               [("dr_col", C.POINTER(C.c_double)), ("dz_row", C.POINTER(C.c_double))]


class Material(C.Structure):
    _fields_ = [(n, C.c_double) for n in ("rho0", "A", "B", "E0", "a", "b", "alpha", "beta", "Eiv", "Ecv",
                                          "p_min", "c_floor_frac")] + \
               [("strength", C.c_int32), ("damage", C.c_int32)] + \
               [(n, C.c_double) for n in ("Y0", "mu_f", "Ylim", "poisson", "Yd0", "mu_d", "Ydm", "eps_fb",
                                          "B_dmg", "p_bd", "gamma_eta", "gamma_T", "c_vib", "af_h")]


class PmlC(C.Structure):
    _fields_ = [("enabled", C.c_int32), ("damp_stress", C.c_int32), ("R", C.c_double), ("c_ref", C.c_double),
                ("placement", C.c_int32), ("reserved", C.c_int32)]


class SceneC(C.Structure):
    _fields_ = [("surface_j", C.c_int32), ("subsample", C.c_int32), ("radius", C.c_double),
                ("v_imp", C.c_double), ("gravity", C.c_double), ("layer_j", C.c_int32),
                ("layer2_j", C.c_int32)]


_DP = C.POINTER(C.c_double)


class Fields(C.Structure):
    _fields_ = [(n, _DP) for n in ("rho", "I", "f", "s", "v", "p", "c2")]


class Diag(C.Structure):
    _fields_ = [("t", C.c_double), ("dt", C.c_double), ("dt_prev", C.c_double), ("cycle", C.c_int64),
                ("mass", C.c_double), ("ie", C.c_double), ("ke", C.c_double), ("mass_out", C.c_double),
                ("mass_pml", C.c_double), ("ie_out", C.c_double), ("err", C.c_int32),
                ("err_cycle", C.c_int32)]


class Instance(C.Structure):
    _fields_ = [("grid", Grid), ("mats", Material * 3), ("pml", PmlC), ("scene", SceneC),
                ("has_scene", C.c_int32), ("reserved", C.c_int32)]


class Schedule(C.Structure):
    _fields_ = [("variant", C.c_int32), ("tile_r", C.c_int32), ("tile_z", C.c_int32), ("threads", C.c_int32),
                ("grid", C.c_int32), ("reserved", C.c_int32), ("ms_per_cycle", C.c_double)]


_lib = None


def load() -> C.CDLL:
    """Load libsalec.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"libsalec.so not built ({LIB_PATH}); run __graft_entry__.build()")
    # torch first: the library must bind to the HIP runtime torch loads (a
    # process whose first HIP runtime came with libsalec sees no device from
    # it once torch has initialised its own)
    import torch  # noqa: F401
    lib = C.CDLL(LIB_PATH)
    P = C.c_void_p
    I32 = C.c_int32
    lib.salec_plan.restype = C.c_size_t
    lib.salec_plan.argtypes = [C.POINTER(Grid), C.POINTER(Material), C.POINTER(PmlC)]
    lib.salec_plan_batch.restype = C.c_size_t
    lib.salec_plan_batch.argtypes = [C.POINTER(Instance), I32]
    lib.salec_init.argtypes = [C.POINTER(Grid), C.POINTER(Material), C.POINTER(PmlC), C.POINTER(SceneC),
                               P, C.c_size_t, P, C.POINTER(P)]
    lib.salec_init_batch.argtypes = [C.POINTER(Instance), I32, P, C.c_size_t, P, C.POINTER(P)]
    lib.salec_num_instances.restype = I32
    lib.salec_num_instances.argtypes = [P]
    lib.salec_step.argtypes = [P, I32]
    lib.salec_enqueue.argtypes = [P, I32]
    lib.salec_get_fields.argtypes = [P, I32, C.POINTER(Fields)]
    lib.salec_set_fields.argtypes = [P, I32, C.POINTER(Fields)]
    lib.salec_get_pml.argtypes = [P, I32, _DP, _DP]
    lib.salec_set_pml.argtypes = [P, I32, _DP, _DP]
    lib.salec_set_clock.argtypes = [P, I32, C.c_double, C.c_double]
    lib.salec_state_bytes.restype = C.c_size_t
    lib.salec_state_bytes.argtypes = [P]
    lib.salec_get_state.argtypes = [P, P, C.c_size_t]
    lib.salec_set_state.argtypes = [P, P, C.c_size_t]
    lib.salec_diag.argtypes = [P, I32, C.POINTER(Diag)]
    lib.salec_diag_totals.argtypes = [P, I32, P]
    lib.salec_last_step_ms.argtypes = [P, _DP]
    lib.salec_time_kernels.argtypes = [P, I32, _DP, _DP]
    lib.salec_set_p0.argtypes = [P, I32, _DP]
    lib.salec_get_p0.argtypes = [P, I32, _DP]
    lib.salec_set_materials.argtypes = [P, I32, _DP, _DP]
    lib.salec_get_materials.argtypes = [P, I32, _DP, _DP]
    lib.salec_set_damage.argtypes = [P, I32, _DP, _DP]
    lib.salec_get_damage.argtypes = [P, I32, _DP, _DP]
    lib.salec_num_variants.restype = I32
    lib.salec_num_variants.argtypes = []
    lib.salec_get_schedule.argtypes = [P, C.POINTER(Schedule)]
    lib.salec_set_schedule.argtypes = [P, I32, I32]
    lib.salec_tune.argtypes = [P, I32, C.POINTER(Schedule)]
    lib.salec_last_error.restype = C.c_char_p
    lib.salec_last_error.argtypes = [P]
    lib.salec_destroy.argtypes = [P]
    _lib = lib
    return lib


def header_functions() -> list:
    """Names of the functions include/salec.h declares."""
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(salec_[a-z_0-9]+)\s*\(", txt)))


def _grid(g, precision, keep: list) -> Grid:
    """The C grid description; a stretched grid's width / height arrays go
    into `keep`, which the caller holds until the library has read them."""
    drc = None if g.dr_col is None else np.ascontiguousarray(g.dr_col, dtype=np.float64)
    dzr = None if g.dz_row is None else np.ascontiguousarray(g.dz_row, dtype=np.float64)
    keep.extend([drc, dzr])
    return Grid(g.n_r, g.n_z, g.pml_r, g.pml_b, g.nmat, g.top_closed,
                SALEC_MIXED if precision == "mixed" else SALEC_FP64, int(g.closure),
                g.dr, g.dz, g.cfl, g.dt_grow, g.dt_max, g.dt_floor, g.t_stop, g.q_lin, g.q_quad,
                _ptr(drc), _ptr(dzr))


def _mat(m) -> Material:
    return Material(m.rho0, m.A, m.B, m.E0, m.a, m.b, m.alpha, m.beta, m.Eiv, m.Ecv, m.p_min,
                    m.c_floor_frac, int(m.strength), int(m.damage), m.Y0, m.mu_f, m.Ylim, m.poisson,
                    m.Yd0, m.mu_d, m.Ydm, m.eps_fb, m.B_dmg, m.p_bd, m.gamma_eta, m.gamma_T, m.c_vib, m.af_h)


def _mats(problem):
    arr = (Material * 3)()
    for k, m in enumerate(problem.mats[:problem.grid.nmat]):
        arr[k] = _mat(m)
    return arr


def _instance(problem, keep: list) -> Instance:
    g = problem.grid
    inst = Instance()
    inst.grid = _grid(g, problem.precision, keep)
    for k, m in enumerate(problem.mats[:g.nmat]):
        inst.mats[k] = _mat(m)
    p = problem.pml
    if int(getattr(p, "form", 0)) != 0:
        raise ValueError("the library damps the specific velocity and energy (pml.form = 0)")
    inst.pml = PmlC(int(p.enabled), int(p.damp_stress), p.R, p.c_ref, int(getattr(p, "placement", 0)), 0)
    if problem.scene is not None:
        sc = problem.scene
        inst.scene = SceneC(sc.surface_j, sc.subsample, sc.radius, sc.v_imp, sc.gravity, sc.layer_j,
                             sc.layer2_j)
        inst.has_scene = 1
    return inst


def plan_bytes(problems) -> int:
    """Device bytes for one problem or a list of problems (an ensemble)."""
    lib = load()
    probs = problems if isinstance(problems, (list, tuple)) else [problems]
    keep = []
    arr = (Instance * len(probs))(*[_instance(pb, keep) for pb in probs])
    return lib.salec_plan_batch(arr, len(probs))


def num_variants() -> int:
    return load().salec_num_variants()


def _ptr(a):
    return None if a is None else a.ctypes.data_as(_DP)


class SalecError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{ERRORS.get(code, code)}: {msg}")
        self.code = code


class Salec:
    """A simulation context on a HIP device: one problem, or a list of
    problems advanced together as an ensemble (member k is `problems[k]`)."""

    def __init__(self, problems, device: str = "cuda:0"):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("libsalec needs a HIP device; none is visible")
        lib = load()
        self.lib = lib
        self.problems = list(problems) if isinstance(problems, (list, tuple)) else [problems]
        self.problem = self.problems[0]
        self.dims = []
        for pb in self.problems:
            g = pb.grid
            NR, NZ = g.n_r + g.pml_r, g.n_z + g.pml_b
            self.dims.append((NR, NZ, g.nmat))
        self.NR, self.NZ, self.nmat = self.dims[0]
        self.NC, self.NN = self.NR * self.NZ, (self.NR + 1) * (self.NZ + 1)
        self.device = torch.device(device)
        keep = []
        arr = (Instance * len(self.problems))(*[_instance(pb, keep) for pb in self.problems])
        nbytes = lib.salec_plan_batch(arr, len(self.problems))
        if nbytes == 0:
            raise ValueError("salec_plan_batch rejected the problem description")
        with torch.cuda.device(self.device):
            self.buf = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
            base = self.buf.data_ptr()
            off = (-base) % 256
            # a stream of our own (default priority): the legacy null stream
            # cannot be captured into HIP graphs
            self.stream = torch.cuda.Stream(device=self.device)
        h = C.c_void_p()
        rc = lib.salec_init_batch(arr, len(self.problems), C.c_void_p(base + off), C.c_size_t(nbytes),
                                  C.c_void_p(self.stream.cuda_stream), C.byref(h))
        self._h = h
        if rc:
            msg = lib.salec_last_error(h).decode() if h else ""
            raise SalecError(rc, msg)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            self.lib.salec_destroy(h)
            self._h = None

    def _check(self, rc):
        if rc:
            raise SalecError(rc, self.lib.salec_last_error(self._h).decode())

    @property
    def num_instances(self) -> int:
        return self.lib.salec_num_instances(self._h)

    def step(self, n: int, check: bool = True) -> int:
        rc = self.lib.salec_step(self._h, int(n))
        if rc and check:
            self._check(rc)
        return rc

    def enqueue(self, n: int):
        self._check(self.lib.salec_enqueue(self._h, int(n)))

    def last_step_ms(self) -> float:
        v = C.c_double()
        self._check(self.lib.salec_last_step_ms(self._h, C.byref(v)))
        return v.value

    def time_kernels(self, n: int) -> tuple:
        """Advances n cycles with the two kernels of each cycle launched
        between HIP events; returns their mean durations (cycle kernel,
        finalize kernel) in milliseconds."""
        a, b = C.c_double(), C.c_double()
        self._check(self.lib.salec_time_kernels(self._h, int(n), C.byref(a), C.byref(b)))
        return a.value, b.value

    def fields(self, eos: bool = True, k: int = 0) -> dict:
        NR, NZ, nmat = self.dims[k]
        NC, NN = NR * NZ, (NR + 1) * (NZ + 1)
        rho, I = np.empty(NC), np.empty(NC)
        f, s, v = np.empty(nmat * NC), np.empty(3 * NC), np.empty(2 * NN)
        p = np.empty(NC) if eos else None
        c2 = np.empty(NC) if eos else None
        fl = Fields(_ptr(rho), _ptr(I), _ptr(f), _ptr(s), _ptr(v), _ptr(p), _ptr(c2))
        self._check(self.lib.salec_get_fields(self._h, int(k), C.byref(fl)))
        out = {"rho": rho.reshape(NZ, NR), "I": I.reshape(NZ, NR), "f": f.reshape(nmat, NZ, NR),
               "s": s.reshape(3, NZ, NR), "v": v.reshape(2, NZ + 1, NR + 1)}
        if eos:
            out["p"] = p.reshape(NZ, NR)
            out["c2"] = c2.reshape(NZ, NR)
        return out

    def fractions(self, k: int = 0):
        """Volume fractions of member k only, (nmat, NZ, NR)."""
        NR, NZ, nmat = self.dims[k]
        f = np.empty(nmat * NR * NZ)
        fl = Fields(None, None, _ptr(f), None, None, None, None)
        self._check(self.lib.salec_get_fields(self._h, int(k), C.byref(fl)))
        return f.reshape(nmat, NZ, NR)

    def set_fields(self, rho, I, f, v, s=None, k: int = 0):
        NR, NZ, nmat = self.dims[k]
        NC, NN = NR * NZ, (NR + 1) * (NZ + 1)
        arr = [np.ascontiguousarray(a, dtype=np.float64).reshape(-1) for a in (rho, I, f, v)]
        if not (arr[0].size == NC and arr[1].size == NC and arr[2].size == nmat * NC and arr[3].size == 2 * NN):
            raise ValueError("field shapes do not match the instance")
        sp = None if s is None else np.ascontiguousarray(s, dtype=np.float64).reshape(3 * NC)
        fl = Fields(_ptr(arr[0]), _ptr(arr[1]), _ptr(arr[2]), _ptr(sp), _ptr(arr[3]), None, None)
        self._check(self.lib.salec_set_fields(self._h, int(k), C.byref(fl)))

    def set_p0(self, p0, k: int = 0):
        """Initial pressure per cell row (NZ values, Pa) of member k."""
        NR, NZ, _ = self.dims[k]
        p0 = np.ascontiguousarray(p0, dtype=np.float64).reshape(NZ)
        self._check(self.lib.salec_set_p0(self._h, int(k), _ptr(p0)))

    def p0(self, k: int = 0):
        NR, NZ, _ = self.dims[k]
        out = np.empty(NZ)
        self._check(self.lib.salec_get_p0(self._h, int(k), _ptr(out)))
        return out

    def set_materials(self, mu, Im, k: int = 0):
        """Per-material state of member k (per-material closure): partial
        densities and specific energies, each (nmat, NZ, NR)."""
        NR, NZ, nmat = self.dims[k]
        mu = np.ascontiguousarray(mu, dtype=np.float64).reshape(nmat * NZ * NR)
        Im = np.ascontiguousarray(Im, dtype=np.float64).reshape(nmat * NZ * NR)
        self._check(self.lib.salec_set_materials(self._h, int(k), _ptr(mu), _ptr(Im)))

    def materials(self, k: int = 0) -> dict:
        """{"mu": partial densities, "Im": specific energies}, (nmat, NZ, NR)."""
        NR, NZ, nmat = self.dims[k]
        mu, Im = np.empty(nmat * NZ * NR), np.empty(nmat * NZ * NR)
        self._check(self.lib.salec_get_materials(self._h, int(k), _ptr(mu), _ptr(Im)))
        return {"mu": mu.reshape(nmat, NZ, NR), "Im": Im.reshape(nmat, NZ, NR)}

    def set_damage(self, D=None, vib=None, k: int = 0):
        """Damage and block-model vibration speed of member k, each (NZ, NR);
        None keeps that field. Starts a new run from the current state."""
        NR, NZ, _ = self.dims[k]
        Dp = None if D is None else np.ascontiguousarray(D, dtype=np.float64).reshape(NZ * NR)
        Vp = None if vib is None else np.ascontiguousarray(vib, dtype=np.float64).reshape(NZ * NR)
        self._check(self.lib.salec_set_damage(self._h, int(k), _ptr(Dp), _ptr(Vp)))

    def damage(self, k: int = 0) -> dict:
        """{"D": damage, "vib": vibration speed}, (NZ, NR) each."""
        NR, NZ, _ = self.dims[k]
        D, V = np.empty(NZ * NR), np.empty(NZ * NR)
        self._check(self.lib.salec_get_damage(self._h, int(k), _ptr(D), _ptr(V)))
        return {"D": D.reshape(NZ, NR), "vib": V.reshape(NZ, NR)}

    @property
    def has_damage(self) -> bool:
        return any(int(m.damage) for pb in self.problems for m in pb.mats[:pb.grid.nmat])

    def pml_aux(self, k: int = 0) -> dict:
        NR, NZ, _ = self.dims[k]
        NC, NN = NR * NZ, (NR + 1) * (NZ + 1)
        ca, na = np.empty(8 * NC), np.empty(8 * NN)
        self._check(self.lib.salec_get_pml(self._h, int(k), _ptr(ca), _ptr(na)))
        ca, na = ca.reshape(8, NZ, NR), na.reshape(8, NZ + 1, NR + 1)
        names_c = ["phi1_b", "phi3_b", "psi2_b", "phi1_r", "phi3_r", "psi2_r", "rho_ref", "msink"]
        names_n = ["phi2_b_r", "phi2_b_z", "psi1_b_r", "psi1_b_z", "phi2_r_r", "phi2_r_z", "psi1_r_r",
                   "psi1_r_z"]
        out = {n: ca[i] for i, n in enumerate(names_c)}
        out.update({n: na[i] for i, n in enumerate(names_n)})
        return out

    def set_pml(self, aux: dict, k: int = 0):
        """Writes member k's PML auxiliaries back in the layout pml_aux returns."""
        NR, NZ, _ = self.dims[k]
        names_c = ["phi1_b", "phi3_b", "psi2_b", "phi1_r", "phi3_r", "psi2_r", "rho_ref", "msink"]
        names_n = ["phi2_b_r", "phi2_b_z", "psi1_b_r", "psi1_b_z", "phi2_r_r", "phi2_r_z", "psi1_r_r",
                   "psi1_r_z"]
        ca = np.ascontiguousarray(np.stack([np.asarray(aux[n], dtype=np.float64).reshape(NZ, NR)
                                            for n in names_c]))
        na = np.ascontiguousarray(np.stack([np.asarray(aux[n], dtype=np.float64).reshape(NZ + 1, NR + 1)
                                            for n in names_n]))
        self._check(self.lib.salec_set_pml(self._h, int(k), _ptr(ca.reshape(-1)), _ptr(na.reshape(-1))))

    def set_clock(self, t: float, dt: float, k: int = 0):
        """Time of member k and the step of its next cycle."""
        self._check(self.lib.salec_set_clock(self._h, int(k), float(t), float(dt)))

    def continue_from(self, src: "Salec", k_src: int = 0, k: int = 0):
        """Member k takes over member k_src of context src between cycles:
        fields, per-material state, PML auxiliaries and clock, each in this
        context's precision. The problems must be the same up to precision."""
        F = src.fields(eos=False, k=k_src)
        self.set_fields(F["rho"], F["I"], F["f"], F["v"], F["s"], k=k)
        if self.problems[k].grid.closure:
            M = src.materials(k=k_src)
            self.set_materials(M["mu"], M["Im"], k=k)
        if self.has_damage:
            Dm = src.damage(k=k_src)
            self.set_damage(Dm["D"], Dm["vib"], k=k)
        self.set_pml(src.pml_aux(k=k_src), k=k)
        d = src.diag(k=k_src)
        self.set_clock(d["t"], d["dt"], k=k)

    def diag(self, k: int = 0) -> dict:
        d = Diag()
        self._check(self.lib.salec_diag(self._h, int(k), C.byref(d)))
        return {n: getattr(d, n) for n, _ in Diag._fields_}

    def diag_totals(self, out, k: int = 0):
        """Enqueues member k's compensated totals (mass, ie, ke, mass_out,
        mass_pml, ie_out) into `out`, a float64 tensor of >= 6 values on the
        context's device, on the context's stream (no allocation, no
        synchronisation: wait on self.stream before reading)."""
        if not out.dtype.is_floating_point or out.element_size() != 8 or out.numel() < 6 or not out.is_cuda \
                or not out.is_contiguous():
            raise ValueError("out must be a contiguous float64 device tensor of at least 6 values")
        self._check(self.lib.salec_diag_totals(self._h, int(k), C.c_void_p(out.data_ptr())))

    def get_state(self) -> bytes:
        n = self.lib.salec_state_bytes(self._h)
        buf = C.create_string_buffer(n)
        self._check(self.lib.salec_get_state(self._h, buf, n))
        return buf.raw

    def set_state(self, blob: bytes):
        buf = C.create_string_buffer(blob, len(blob))
        self._check(self.lib.salec_set_state(self._h, buf, len(blob)))

    def schedule(self) -> dict:
        s = Schedule()
        self._check(self.lib.salec_get_schedule(self._h, C.byref(s)))
        return {n: getattr(s, n) for n, _ in Schedule._fields_}

    def set_schedule(self, variant: int, grid: int = 0):
        self._check(self.lib.salec_set_schedule(self._h, int(variant), int(grid)))

    def tune(self, cycles: int) -> dict:
        s = Schedule()
        self._check(self.lib.salec_tune(self._h, int(cycles), C.byref(s)))
        return {n: getattr(s, n) for n, _ in Schedule._fields_}
