"""ctypes binding of the plain FP64 CPU oracle (test infrastructure only).

Only the tests, the smoke check and the benchmark's CPU-baseline leg may use
this module; the product path never imports it. It reads problem
descriptions by attribute (grid, mats, pml, scene) and imports nothing from
the HIP library's package.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsalec_oracle.so")

_lib = None


class _Grid(C.Structure):
    _fields_ = [("n_r", C.c_int32), ("n_z", C.c_int32), ("pml_r", C.c_int32),
                ("pml_b", C.c_int32), ("nmat", C.c_int32), ("top_closed", C.c_int32),
                ("closure", C.c_int32), ("dr", C.c_double), ("dz", C.c_double), ("cfl", C.c_double),
                ("dt_grow", C.c_double), ("dt_max", C.c_double), ("dt_floor", C.c_double),
                ("t_stop", C.c_double), ("q_lin", C.c_double), ("q_quad", C.c_double),
                ("dr_col", C.POINTER(C.c_double)), ("dz_row", C.POINTER(C.c_double))]


class _Mat(C.Structure):
    _fields_ = [(n, C.c_double) for n in ("rho0", "A", "B", "E0", "a", "b", "alpha", "beta",
                                          "Eiv", "Ecv", "p_min", "c_floor_frac")] + \
               [("strength", C.c_int32)] + \
               [(n, C.c_double) for n in ("Y0", "mu_f", "Ylim", "poisson")] + \
               [("damage", C.c_int32)] + \
               [(n, C.c_double) for n in ("Yd0", "mu_d", "Ydm", "eps_fb", "B_dmg", "p_bd",
                                          "gamma_eta", "gamma_T", "c_vib", "af_h")]


class _Pml(C.Structure):
    _fields_ = [("enabled", C.c_int32), ("damp_stress", C.c_int32), ("R", C.c_double), ("c_ref", C.c_double),
                ("placement", C.c_int32), ("form", C.c_int32)]


class _Scene(C.Structure):
    _fields_ = [("surface_j", C.c_int32), ("subsample", C.c_int32), ("radius", C.c_double),
                ("v_imp", C.c_double), ("gravity", C.c_double), ("layer_j", C.c_int32),
                ("layer2_j", C.c_int32)]


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        from . import build as _b  # noqa: F401  (package-relative when imported as oracle.oracle)
        _b.build()
    lib = C.CDLL(LIB_PATH)
    P = C.c_void_p
    D = C.POINTER(C.c_double)
    lib.orc_create.restype = P
    lib.orc_create.argtypes = [C.POINTER(_Grid), C.POINTER(_Mat), C.POINTER(_Pml)]
    lib.orc_destroy.argtypes = [P]
    lib.orc_set_threads.argtypes = [C.c_int]
    lib.orc_set_threads.restype = C.c_int
    lib.orc_init_scene.argtypes = [P, C.POINTER(_Scene)]
    lib.orc_set_fields.argtypes = [P, D, D, D, D, D]
    lib.orc_set_p0.argtypes = [P, D]
    lib.orc_set_materials.argtypes = [P, D, D]
    lib.orc_get_materials.argtypes = [P, D, D]
    lib.orc_get_p0.argtypes = [P, D]
    lib.orc_set_damage.argtypes = [P, D, D]
    lib.orc_get_damage.argtypes = [P, D, D]
    lib.orc_yield_damaged.argtypes = [C.POINTER(_Mat), C.c_double, C.c_double, C.c_double]
    lib.orc_yield_damaged.restype = C.c_double
    lib.orc_failure_strain.argtypes = [C.POINTER(_Mat), C.c_double]
    lib.orc_failure_strain.restype = C.c_double
    lib.orc_step.argtypes = [P, C.c_int32]
    lib.orc_get_fields.argtypes = [P, D, D, D, D, D, D, D]
    lib.orc_get_pml.argtypes = [P, D, D]
    lib.orc_set_pml.argtypes = [P, D, D]
    lib.orc_set_clock.argtypes = [P, C.c_double, C.c_double]
    lib.orc_diag.argtypes = [P, D]
    lib.orc_get_profiles.argtypes = [P, D, D, D, D]
    lib.orc_tillotson.argtypes = [C.POINTER(_Mat), C.c_double, C.c_double, D, D]
    lib.orc_exp.argtypes = [C.c_double]
    lib.orc_exp.restype = C.c_double
    lib.orc_yield.argtypes = [C.POINTER(_Mat), C.c_double]
    lib.orc_yield.restype = C.c_double
    lib.orc_shear_modulus.argtypes = [C.POINTER(_Mat)]
    lib.orc_shear_modulus.restype = C.c_double
    lib.orc_stress_update.argtypes = [C.c_double, C.c_double, C.c_double, D, D]
    lib.orc_cell_kinematics.argtypes = [C.POINTER(_Grid), C.c_int32, C.c_int32, D, D, D]
    lib.orc_get_geometry.argtypes = [P, D, D, D, D]
    _lib = lib
    return lib


def _ptr(a):
    if a is None:
        return None
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _grid(g) -> _Grid:
    """The C grid description; a stretched grid's width / height arrays are
    kept alive on the returned structure for as long as it is used."""
    drc = None if g.dr_col is None else np.ascontiguousarray(g.dr_col, dtype=np.float64)
    dzr = None if g.dz_row is None else np.ascontiguousarray(g.dz_row, dtype=np.float64)
    out = _Grid(g.n_r, g.n_z, g.pml_r, g.pml_b, g.nmat, g.top_closed, g.closure, g.dr, g.dz, g.cfl,
                g.dt_grow, g.dt_max, g.dt_floor, g.t_stop, g.q_lin, g.q_quad, _ptr(drc), _ptr(dzr))
    out._keep = (drc, dzr)
    return out


def _mat(m) -> _Mat:
    return _Mat(m.rho0, m.A, m.B, m.E0, m.a, m.b, m.alpha, m.beta, m.Eiv, m.Ecv, m.p_min,
                m.c_floor_frac, int(m.strength), m.Y0, m.mu_f, m.Ylim, m.poisson,
                int(getattr(m, "damage", 0)), *[float(getattr(m, n, d)) for n, d in (
                    ("Yd0", 0.0), ("mu_d", 0.0), ("Ydm", 0.0), ("eps_fb", 1e-4), ("B_dmg", 1e-11),
                    ("p_bd", 3e8), ("gamma_eta", 0.0), ("gamma_T", 0.0), ("c_vib", 0.0), ("af_h", 0.0))])


def set_threads(n: int) -> int:
    return _load().orc_set_threads(int(n))


class OracleError(RuntimeError):
    def __init__(self, code, cycle):
        super().__init__(f"oracle error {code} at cycle {cycle}")
        self.code = code
        self.cycle = cycle


class Oracle:
    """One simulation instance on the CPU. Arrays are (NZ, NR) for cells and
    (NZ+1, NR+1) for nodes, row-major with r fastest."""

    def __init__(self, problem):
        lib = _load()
        self.problem = problem
        g = problem.grid
        self.g = g
        self.NR, self.NZ = g.n_r + g.pml_r, g.n_z + g.pml_b
        self.NC, self.NN = self.NR * self.NZ, (self.NR + 1) * (self.NZ + 1)
        self.nmat = g.nmat
        mats = (_Mat * 3)(*[_mat(m) for m in problem.mats[:g.nmat]])
        pml = problem.pml
        cp = _Pml(int(pml.enabled), int(pml.damp_stress), pml.R, pml.c_ref, int(getattr(pml, "placement", 0)),
                  int(getattr(pml, "form", 0)))
        self._h = lib.orc_create(C.byref(_grid(g)), mats, C.byref(cp))
        if not self._h:
            raise ValueError("oracle rejected the problem description")
        self._lib = lib
        if problem.scene is not None:
            sc = problem.scene
            rc = lib.orc_init_scene(self._h, C.byref(_Scene(sc.surface_j, sc.subsample, sc.radius, sc.v_imp,
                                                            sc.gravity, sc.layer_j, sc.layer2_j)))
            if rc:
                raise ValueError(f"orc_init_scene failed: {rc}")

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            self._lib.orc_destroy(h)
            self._h = None

    def set_fields(self, rho, I, f, v, s=None):
        NC, NN = self.NC, self.NN
        rho = np.ascontiguousarray(rho, dtype=np.float64).reshape(NC)
        I = np.ascontiguousarray(I, dtype=np.float64).reshape(NC)
        f = np.ascontiguousarray(f, dtype=np.float64).reshape(self.nmat * NC)
        v = np.ascontiguousarray(v, dtype=np.float64).reshape(2 * NN)
        sp = None if s is None else np.ascontiguousarray(s, dtype=np.float64).reshape(3 * NC)
        rc = self._lib.orc_set_fields(self._h, _ptr(rho), _ptr(I), _ptr(f), _ptr(sp), _ptr(v))
        if rc:
            raise ValueError(f"orc_set_fields failed: {rc}")

    def set_p0(self, p0):
        """Initial pressure per cell row (NZ values, Pa)."""
        p0 = np.ascontiguousarray(p0, dtype=np.float64).reshape(self.NZ)
        if self._lib.orc_set_p0(self._h, _ptr(p0)):
            raise ValueError("orc_set_p0 failed")

    def p0(self):
        out = np.empty(self.NZ)
        self._lib.orc_get_p0(self._h, _ptr(out))
        return out

    def set_materials(self, mu, Im):
        """Per-material state (closure 1): partial densities and specific
        energies, each (nmat, NZ, NR)."""
        n = self.nmat * self.NC
        mu = np.ascontiguousarray(mu, dtype=np.float64).reshape(n)
        Im = np.ascontiguousarray(Im, dtype=np.float64).reshape(n)
        if self._lib.orc_set_materials(self._h, _ptr(mu), _ptr(Im)):
            raise ValueError("orc_set_materials failed")

    def materials(self) -> dict:
        """{"mu": partial densities, "Im": specific energies}, (nmat, NZ, NR)."""
        mu, Im = np.empty(self.nmat * self.NC), np.empty(self.nmat * self.NC)
        if self._lib.orc_get_materials(self._h, _ptr(mu), _ptr(Im)):
            raise ValueError("orc_get_materials failed (closure 0)")
        shp = (self.nmat, self.NZ, self.NR)
        return {"mu": mu.reshape(shp), "Im": Im.reshape(shp)}

    def set_damage(self, D=None, vib=None):
        """Damage and block-model vibration speed per cell (NZ x NR each)."""
        a = None if D is None else np.ascontiguousarray(D, dtype=np.float64).reshape(-1)
        b = None if vib is None else np.ascontiguousarray(vib, dtype=np.float64).reshape(-1)
        for x in (a, b):
            if x is not None and x.size != self.NC:
                raise ValueError("damage arrays must have NZ x NR values")
        rc = self._lib.orc_set_damage(self._h, _ptr(a), _ptr(b))
        if rc:
            raise ValueError(rc)

    def damage(self) -> dict:
        D, vib = np.empty(self.NC), np.empty(self.NC)
        self._lib.orc_get_damage(self._h, _ptr(D), _ptr(vib))
        return {"D": D.reshape(self.NZ, self.NR), "vib": vib.reshape(self.NZ, self.NR)}

    def step(self, n: int, check: bool = True) -> int:
        rc = self._lib.orc_step(self._h, int(n))
        if rc and check:
            d = self.diag()
            raise OracleError(rc, int(d["err_cycle"]))
        return rc

    def fields(self, eos: bool = True) -> dict:
        NR, NZ, NC, NN = self.NR, self.NZ, self.NC, self.NN
        rho = np.empty(NC)
        I = np.empty(NC)
        f = np.empty(self.nmat * NC)
        s = np.empty(3 * NC)
        v = np.empty(2 * NN)
        p = np.empty(NC) if eos else None
        c2 = np.empty(NC) if eos else None
        self._lib.orc_get_fields(self._h, _ptr(rho), _ptr(I), _ptr(f), _ptr(s), _ptr(v), _ptr(p), _ptr(c2))
        out = {"rho": rho.reshape(NZ, NR), "I": I.reshape(NZ, NR),
               "f": f.reshape(self.nmat, NZ, NR), "s": s.reshape(3, NZ, NR),
               "v": v.reshape(2, NZ + 1, NR + 1)}
        if eos:
            out["p"] = p.reshape(NZ, NR)
            out["c2"] = c2.reshape(NZ, NR)
        return out

    def pml_aux(self) -> dict:
        NR, NZ, NC, NN = self.NR, self.NZ, self.NC, self.NN
        ca = np.empty(8 * NC)
        na = np.empty(8 * NN)
        self._lib.orc_get_pml(self._h, _ptr(ca), _ptr(na))
        ca = ca.reshape(8, NZ, NR)
        na = na.reshape(8, NZ + 1, NR + 1)
        names_c = ["phi1_b", "phi3_b", "psi2_b", "phi1_r", "phi3_r", "psi2_r", "rho_ref", "msink"]
        names_n = ["phi2_b_r", "phi2_b_z", "psi1_b_r", "psi1_b_z", "phi2_r_r", "phi2_r_z",
                   "psi1_r_r", "psi1_r_z"]
        out = {k: ca[i] for i, k in enumerate(names_c)}
        out.update({k: na[i] for i, k in enumerate(names_n)})
        return out

    def set_pml(self, aux: dict):
        """Writes the PML auxiliaries back in the layout pml_aux returns."""
        names_c = ["phi1_b", "phi3_b", "psi2_b", "phi1_r", "phi3_r", "psi2_r", "rho_ref", "msink"]
        names_n = ["phi2_b_r", "phi2_b_z", "psi1_b_r", "psi1_b_z", "phi2_r_r", "phi2_r_z",
                   "psi1_r_r", "psi1_r_z"]
        ca = np.ascontiguousarray(np.stack([np.asarray(aux[k], dtype=np.float64).reshape(self.NZ, self.NR)
                                            for k in names_c])).reshape(-1)
        na = np.ascontiguousarray(np.stack([np.asarray(aux[k], dtype=np.float64).reshape(self.NZ + 1, self.NR + 1)
                                            for k in names_n])).reshape(-1)
        if self._lib.orc_set_pml(self._h, _ptr(ca), _ptr(na)):
            raise ValueError("orc_set_pml failed")

    def set_clock(self, t: float, dt: float):
        if self._lib.orc_set_clock(self._h, float(t), float(dt)):
            raise ValueError("orc_set_clock: needs t >= 0 and 0 < dt <= dt_max (and dt <= t_stop - t)")

    def continue_from(self, src: "Oracle"):
        """Takes over src's state between cycles: fields, per-material state,
        PML auxiliaries and clock. The problems must be the same."""
        F = src.fields(eos=False)
        self.set_fields(F["rho"], F["I"], F["f"], F["v"], F["s"])
        if self.problem.grid.closure:
            M = src.materials()
            self.set_materials(M["mu"], M["Im"])
        self.set_pml(src.pml_aux())
        d = src.diag()
        self.set_clock(d["t"], d["dt"])

    def geometry(self):
        """Node and centre radii and heights of the grid."""
        rn, rc = np.empty(self.NR + 1), np.empty(self.NR)
        zn, zc = np.empty(self.NZ + 1), np.empty(self.NZ)
        self._lib.orc_get_geometry(self._h, _ptr(rn), _ptr(rc), _ptr(zn), _ptr(zc))
        return rn, rc, zn, zc

    def profiles(self):
        dcz, dnz = np.empty(self.NZ), np.empty(self.NZ + 1)
        dcr, dnr = np.empty(self.NR), np.empty(self.NR + 1)
        self._lib.orc_get_profiles(self._h, _ptr(dcz), _ptr(dnz), _ptr(dcr), _ptr(dnr))
        return dcz, dnz, dcr, dnr

    def diag(self) -> dict:
        out = np.empty(12)
        self._lib.orc_diag(self._h, _ptr(out))
        keys = ["t", "dt", "cycle", "mass", "ie", "ke", "mass_out", "mass_pml", "ie_out",
                "err", "err_cycle", "dt_prev"]
        return dict(zip(keys, out.tolist()))


# ---- point functions ----------------------------------------------------
def exp(x: float) -> float:
    return _load().orc_exp(float(x))


def tillotson(mat, rho: float, e: float):
    p, c2 = C.c_double(), C.c_double()
    _load().orc_tillotson(C.byref(_mat(mat)), float(rho), float(e), C.byref(p), C.byref(c2))
    return p.value, c2.value


def yield_strength(mat, p: float) -> float:
    return _load().orc_yield(C.byref(_mat(mat)), float(p))


def yield_damaged(mat, p: float, D: float, p_vib: float) -> float:
    return _load().orc_yield_damaged(C.byref(_mat(mat)), float(p), float(D), float(p_vib))


def failure_strain(mat, p: float) -> float:
    return _load().orc_failure_strain(C.byref(_mat(mat)), float(p))


def shear_modulus(mat) -> float:
    return _load().orc_shear_modulus(C.byref(_mat(mat)))


def stress_update(G: float, Y: float, dt: float, rates, s):
    r = np.ascontiguousarray(rates, dtype=np.float64)
    s = np.array(s, dtype=np.float64)
    _load().orc_stress_update(float(G), float(Y), float(dt), _ptr(r), _ptr(s))
    return s


def cell_kinematics(grid, i: int, vr4, vz4, j: int = 0):
    vr = np.ascontiguousarray(vr4, dtype=np.float64)
    vz = np.ascontiguousarray(vz4, dtype=np.float64)
    out = np.empty(6)
    cg = _grid(grid)
    _load().orc_cell_kinematics(C.byref(cg), int(i), int(j), _ptr(vr), _ptr(vz), _ptr(out))
    return dict(zip(["err", "ezz", "ett", "erz", "om", "D"], out.tolist()))
