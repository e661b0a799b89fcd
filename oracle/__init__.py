"""CPU oracle for the explicit 1D3V PIC/MCC step (arXiv:2109.04469, Sec. 2).

TEST INFRASTRUCTURE ONLY: imported by tests/, by __graft_entry__.smoke()
and by the CPU-baseline leg of bench.py, never by the simulation package.
The step's arithmetic lives in plain C (pic_oracle.c, philox.c,
warm_oracle.c); this module builds that library with gcc and marshals numpy
arrays to it, and writes out in numpy the few closed-form diagnostics derived
from its averages (monitors) and the warm-start network (mlp.py).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle.so")
OMP_PATH = os.path.join(HERE, "liboracle_omp.so")
SOURCES = [os.path.join(HERE, "pic_oracle.c"), os.path.join(HERE, "philox.c"),
           os.path.join(HERE, "warm_oracle.c")]
CFLAGS = ["-O2", "-std=gnu11", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared"]

NCOUNTERS = 16
F_NO_FIELD, F_FIXED_E, F_NO_COLL, F_IMMOBILE_IONS, F_RECORD = 1, 2, 4, 8, 16


def build(force=True, extra_flags=(), openmp=True):
    """Compile liboracle.so with gcc (FP contraction off, no fast-math) and,
    with openmp, the same sources with -fopenmp as liboracle_omp.so (a pass
    split over threads in slot-ordered runs; used only to time the oracle
    on several cores)."""
    _compile(LIB_PATH, force, extra_flags)
    if openmp:
        _compile(OMP_PATH, force, ("-fopenmp", *extra_flags))
    return LIB_PATH


def _compile(path, force, flags):
    if not force and os.path.exists(path):
        newest = max(os.path.getmtime(s) for s in SOURCES)
        if os.path.getmtime(path) >= newest:
            return
    tmp = path + ".tmp%d" % os.getpid()
    cmd = ["gcc", *CFLAGS, *flags, "-o", tmp, *SOURCES, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, path)


_lib = None
_lib_omp = None


def lib():
    """The plain single-threaded oracle (the checker)."""
    global _lib
    if _lib is None:
        _compile(LIB_PATH, False, ())
        _lib = _declare(ctypes.CDLL(LIB_PATH))
    return _lib


def lib_openmp():
    """The OpenMP build of the same sources (timing only); its thread count
    follows OMP_NUM_THREADS, read when the library is first loaded."""
    global _lib_omp
    if _lib_omp is None:
        _compile(OMP_PATH, False, ("-fopenmp",))
        _lib_omp = _declare(ctypes.CDLL(OMP_PATH))
    return _lib_omp


def threads(openmp=False):
    return int((lib_openmp() if openmp else lib()).ora_threads())


def _declare(L):
    """Argument and result types of the library's entry points."""
    P = ctypes.c_void_p
    d = ctypes.POINTER(ctypes.c_double)
    i64p = ctypes.POINTER(ctypes.c_int64)
    u32p = ctypes.POINTER(ctypes.c_uint32)
    u64p = ctypes.POINTER(ctypes.c_uint64)
    L.ora_philox4x32_10.argtypes = [u32p, u32p, u32p]
    L.ora_philox4x64_10.argtypes = [u64p, u64p, u64p]
    L.ora_create.restype = P
    L.ora_create.argtypes = [ctypes.POINTER(OraParams), d, d, d, d, d]
    L.ora_free.argtypes = [P]
    L.ora_set_state.argtypes = [P, ctypes.c_int, d, d, d, d, ctypes.c_int64, ctypes.c_int64]
    L.ora_get_count.argtypes = [P, ctypes.c_int]
    L.ora_get_count.restype = ctypes.c_int64
    L.ora_get_step.argtypes = [P]
    L.ora_get_step.restype = ctypes.c_int64
    L.ora_get_state.argtypes = [P, ctypes.c_int, d, d, d, d]
    L.ora_set_field.argtypes = [P, d]
    L.ora_get_field.argtypes = [P, d, d, d, i64p, i64p]
    L.ora_get_counters.argtypes = [P, i64p]
    L.ora_get_decisions.argtypes = [P, ctypes.c_int, ctypes.POINTER(ctypes.c_uint8)]
    L.ora_get_decisions.restype = ctypes.c_int64
    L.ora_get_derived.argtypes = [P, d]
    L.ora_measure.argtypes = [P, ctypes.c_int]
    L.ora_moments.argtypes = [P, d, d, d, d, i64p, ctypes.c_int]
    L.ora_step.argtypes = [P, ctypes.c_int64]
    L.ora_step.restype = ctypes.c_int
    L.ora_deposit.argtypes = [P]
    L.ora_solve_field.argtypes = [P]
    L.ora_cell.argtypes = [ctypes.c_int32, ctypes.c_double, ctypes.c_double, i64p, d, i64p]
    L.ora_deposit_array.argtypes = [ctypes.c_int32, ctypes.c_double, ctypes.c_int64, d, i64p]
    L.ora_thomas.argtypes = [ctypes.c_int64, d, d, d, d, d]
    L.ora_poisson.argtypes = [ctypes.c_int32, ctypes.c_double, ctypes.c_double, d, d]
    L.ora_efield.argtypes = [ctypes.c_int32, ctypes.c_double, d, d, d]
    L.ora_wall_raw.argtypes = [P, i64p, i64p, d, i64p, i64p, i64p, d]
    L.ora_load_profile.argtypes = [d, d, ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                   ctypes.c_uint32, ctypes.c_uint32, ctypes.c_int,
                                   ctypes.c_int64, d, d, d, d]
    L.ora_load_profile.restype = ctypes.c_int
    L.ora_threads.restype = ctypes.c_int
    return L


class OraParams(ctypes.Structure):
    _fields_ = [
        ("gap_m", ctypes.c_double), ("pressure_pa", ctypes.c_double),
        ("gas_temp_k", ctypes.c_double), ("rf_voltage_v", ctypes.c_double),
        ("rf_freq_hz", ctypes.c_double),
        ("steps_per_cycle", ctypes.c_int32), ("n_cells", ctypes.c_int32),
        ("weight", ctypes.c_double), ("area_m2", ctypes.c_double),
        ("reflection", ctypes.c_double), ("gamma_see", ctypes.c_double),
        ("see_temp_ev", ctypes.c_double),
        ("capacity", ctypes.c_int64 * 2),
        ("ion_subcycle", ctypes.c_int32), ("sort_interval", ctypes.c_int32),
        ("seed", ctypes.c_uint32), ("run", ctypes.c_uint32),
        ("eepf_bins", ctypes.c_int32),
        ("eepf_emax_ev", ctypes.c_double), ("eepf_halfwidth_m", ctypes.c_double),
        ("flags", ctypes.c_uint32),
        ("ntab", ctypes.c_int32),
        ("dv_e", ctypes.c_double), ("dv_i", ctypes.c_double),
        ("exc_threshold_ev", ctypes.c_double), ("ion_threshold_ev", ctypes.c_double),
    ]


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _ip(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))


def philox4x32_10(ctr, key):
    """Philox4x32-10 block for counter (4 x u32) and key (2 x u32)."""
    L = lib()
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    o = np.zeros(4, dtype=np.uint32)
    p = ctypes.POINTER(ctypes.c_uint32)
    L.ora_philox4x32_10(c.ctypes.data_as(p), k.ctypes.data_as(p), o.ctypes.data_as(p))
    return o


def philox4x64_10(ctr, key):
    L = lib()
    c = np.ascontiguousarray(ctr, dtype=np.uint64)
    k = np.ascontiguousarray(key, dtype=np.uint64)
    o = np.zeros(4, dtype=np.uint64)
    p = ctypes.POINTER(ctypes.c_uint64)
    L.ora_philox4x64_10(c.ctypes.data_as(p), k.ctypes.data_as(p), o.ctypes.data_as(p))
    return o


def cell(nx, inv_dx, x):
    j = ctypes.c_int64()
    f = ctypes.c_double()
    w1 = ctypes.c_int64()
    lib().ora_cell(nx, inv_dx, float(x), ctypes.byref(j), ctypes.byref(f), ctypes.byref(w1))
    return j.value, f.value, w1.value


def deposit_array(nx, inv_dx, x):
    x = np.ascontiguousarray(x, dtype=np.float64)
    dep = np.zeros(nx, dtype=np.int64)
    lib().ora_deposit_array(nx, inv_dx, x.size, _dp(x), _ip(dep))
    return dep


def thomas(a, b, c, d):
    a, b, c, d = (np.ascontiguousarray(v, dtype=np.float64) for v in (a, b, c, d))
    y = np.zeros_like(d)
    lib().ora_thomas(d.size, _dp(a), _dp(b), _dp(c), _dp(d), _dp(y))
    return y


def poisson(nx, dx, V, rho):
    rho = np.ascontiguousarray(rho, dtype=np.float64)
    phi = np.zeros(nx)
    lib().ora_poisson(nx, dx, V, _dp(rho), _dp(phi))
    return phi


def efield(nx, dx, rho, phi):
    rho = np.ascontiguousarray(rho, dtype=np.float64)
    phi = np.ascontiguousarray(phi, dtype=np.float64)
    E = np.zeros(nx)
    lib().ora_efield(nx, dx, _dp(rho), _dp(phi), _dp(E))
    return E


def monitors(moments, params, p_coll):
    """Stability and accuracy monitors of Sec. 3.5 from time averages:
    omega_pe dt with the largest averaged electron density, the Debye length
    sqrt(eps0 T_e / (e n_e)) at L/2 with T_e = (2/3) <eps> (eV), dx / lambda_D
    and the superparticles per Debye length n_e A lambda_D / W at L/2 (the
    middle grid point, or the two middle points combined)."""
    eps0, qe, me = 8.8541878128e-12, 1.602176634e-19, 9.1093837015e-31
    ne = np.asarray(moments["n_e"])
    nx = ne.size
    j0, j1 = (nx - 1) // 2, nx // 2
    nc = 0.5 * (ne[j0] + ne[j1])
    em = np.asarray(moments["mean_energy_e"])
    ec = 0.5 * (em[j0] + em[j1])
    dt = 1.0 / (params["rf_freq_hz"] * params["steps_per_cycle"])
    dx = params["gap_m"] / params["n_cells"]
    lam = np.sqrt(eps0 * (2.0 / 3.0) * ec / (qe * nc)) if nc > 0 else 0.0
    return dict(omega_pe_dt=np.sqrt(ne.max() * qe * qe / (eps0 * me)) * dt, p_coll=tuple(p_coll),
                n_e_max=ne.max(), n_e_center=nc, mean_energy_center_ev=ec, lambda_d_m=lam,
                dx_over_lambda_d=dx / lam if lam > 0 else 0.0,
                n_d=nc * params["area_m2"] * lam / params["weight"])


def load_profile(dens, temp_ev, L, vfac, seed, run, species, n):
    """Particles drawn from a density and a temperature profile on [0, L]
    (warm_oracle.c): returns x, vx, vy, vz."""
    dens = np.ascontiguousarray(dens, dtype=np.float64)
    temp = np.ascontiguousarray(temp_ev, dtype=np.float64)
    assert dens.shape == temp.shape and dens.size >= 2
    out = [np.zeros(int(n)) for _ in range(4)]
    st = lib().ora_load_profile(_dp(dens), _dp(temp), int(dens.size), float(L), float(vfac), int(seed),
                                int(run), int(species), int(n), *[_dp(a) for a in out])
    assert st == 0
    return tuple(out)


class Oracle:
    """One discharge on the CPU oracle. params: a workload parameter dict;
    xs: a pic_inputs.xsec.XsecTables."""

    def __init__(self, params, xs, openmp=False):
        L = lib_openmp() if openmp else lib()
        p = OraParams()
        for name, _ in OraParams._fields_:
            if name in ("ntab", "dv_e", "dv_i", "exc_threshold_ev", "ion_threshold_ev"):
                continue
            v = params[name]
            if name == "capacity":
                p.capacity[0], p.capacity[1] = int(v[0]), int(v[1])
            else:
                setattr(p, name, v)
        p.ntab = xs.n
        p.dv_e = xs.dv_e
        p.dv_i = xs.dv_i
        p.exc_threshold_ev = xs.exc_threshold_ev
        p.ion_threshold_ev = xs.ion_threshold_ev
        self._keep = [np.ascontiguousarray(s, dtype=np.float64) for s in xs.sigma_e + xs.sigma_i]
        self.h = L.ora_create(ctypes.byref(p), *[_dp(a) for a in self._keep])
        if not self.h:
            raise ValueError("oracle rejected the parameter set")
        self.params = dict(params)
        self.nx = int(params["n_cells"]) + 1
        self.L = L

    def __del__(self):
        if getattr(self, "h", None):
            self.L.ora_free(self.h)
            self.h = None

    def set_state(self, species, x, vx, vy, vz, step=0):
        arrs = [np.ascontiguousarray(a, dtype=np.float64) for a in (x, vx, vy, vz)]
        st = self.L.ora_set_state(self.h, species, *[_dp(a) for a in arrs], arrs[0].size, step)
        if st:
            raise RuntimeError("ora_set_state failed: %d" % st)

    def count(self, species):
        return self.L.ora_get_count(self.h, species)

    @property
    def step_index(self):
        return self.L.ora_get_step(self.h)

    def get_state(self, species):
        n = self.count(species)
        arrs = [np.zeros(n) for _ in range(4)]
        self.L.ora_get_state(self.h, species, *[_dp(a) for a in arrs])
        return tuple(arrs)

    def step(self, n=1):
        return self.L.ora_step(self.h, n)

    def set_field(self, E):
        E = np.ascontiguousarray(E, dtype=np.float64)
        assert E.size == self.nx
        self.L.ora_set_field(self.h, _dp(E))

    def deposit(self):
        self.L.ora_deposit(self.h)

    def solve_field(self):
        self.L.ora_solve_field(self.h)

    def get_field(self):
        nx = self.nx
        rho, phi, E = np.zeros(nx), np.zeros(nx), np.zeros(nx)
        de, di = np.zeros(nx, np.int64), np.zeros(nx, np.int64)
        self.L.ora_get_field(self.h, _dp(rho), _dp(phi), _dp(E), _ip(de), _ip(di))
        return dict(rho=rho, phi=phi, E=E, dep_e=de, dep_i=di)

    def counters(self):
        c = np.zeros(NCOUNTERS, np.int64)
        self.L.ora_get_counters(self.h, _ip(c))
        return c

    def decisions(self, species):
        buf = np.zeros(max(1, int(self.params["capacity"][species])), np.uint8)
        n = self.L.ora_get_decisions(self.h, species, buf.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)))
        return buf[:n].copy()

    def derived(self):
        out = np.zeros(8)
        self.L.ora_get_derived(self.h, _dp(out))
        keys = ["dx", "dt", "gas_density", "nu_max_e", "nu_max_i", "p_coll_e", "p_coll_i", "n_x"]
        d = dict(zip(keys, out.tolist()))
        d["n_x"] = int(d["n_x"])
        return d

    def measure(self, on=True):
        self.L.ora_measure(self.h, 1 if on else 0)

    def wall_raw(self):
        """Electrode arrivals since the last moments reset: hits, absorbed,
        energy sums [species, wall], arrival histograms [species, wall, bin],
        ionizations, measured steps and the bins' upper edges per species."""
        nb = int(self.params["eepf_bins"])
        hits = np.zeros(4, np.int64)
        absd = np.zeros(4, np.int64)
        esum = np.zeros(4)
        hist = np.zeros(4 * nb, np.int64)
        ion = ctypes.c_int64()
        st = ctypes.c_int64()
        emax = np.zeros(2)
        self.L.ora_wall_raw(self.h, _ip(hits), _ip(absd), _dp(esum), _ip(hist), ctypes.byref(ion),
                            ctypes.byref(st), _dp(emax))
        return dict(hits=hits.reshape(2, 2), absorbed=absd.reshape(2, 2), esum=esum.reshape(2, 2),
                    hist=hist.reshape(2, 2, nb), ionizations=ion.value, steps=st.value, emax=emax)

    def wall_moments(self):
        """Fluxes per m^2 per s over the measured steps, mean impact energies
        and flux-energy distributions normalised to unit integral (Sec. 3.3)."""
        r = self.wall_raw()
        p = self.params
        dt = 1.0 / (p["rf_freq_hz"] * p["steps_per_cycle"])
        per = p["weight"] / (p["area_m2"] * r["steps"] * dt) if r["steps"] else 0.0
        nb = r["hist"].shape[2]
        fedf = np.zeros((2, 2, nb))
        for k in range(2):
            de = r["emax"][k] / nb
            for w in range(2):
                tot = r["hist"][k, w].sum()
                if tot:
                    fedf[k, w] = r["hist"][k, w] / (tot * de)
        with np.errstate(invalid="ignore", divide="ignore"):
            mean = np.where(r["hits"] > 0, r["esum"] / np.maximum(r["hits"], 1), 0.0)
        return dict(flux=per * r["hits"], absorbed_flux=per * r["absorbed"], mean_energy_ev=mean,
                    fedf=fedf, ionization_rate=per * r["ionizations"], raw=r)

    def moments(self, reset=False):
        nx = self.nx
        ne, ni, em = np.zeros(nx), np.zeros(nx), np.zeros(nx)
        ep = np.zeros(int(self.params["eepf_bins"]))
        st = ctypes.c_int64()
        self.L.ora_moments(self.h, _dp(ne), _dp(ni), _dp(em), _dp(ep), ctypes.byref(st), 1 if reset else 0)
        return dict(n_e=ne, n_i=ni, mean_energy_e=em, eepf=ep, steps=st.value)
