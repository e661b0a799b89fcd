"""Python handle on one simulated discharge. PyTorch provides the device
workspace and the stream; every step of the method runs in libpic's HIP
kernels, reached through the C ABI."""
from __future__ import annotations

import ctypes

import numpy as np
import torch

from . import capi
from .capi import PicDerived, PicMomentsOut, PicParams, PicXsec, check

_PARAM_FIELDS = [f for f, _ in PicParams._fields_]


def make_params(params: dict) -> PicParams:
    p = PicParams()
    for name in _PARAM_FIELDS:
        v = params[name]
        if name == "capacity":
            p.capacity[0], p.capacity[1] = int(v[0]), int(v[1])
        else:
            setattr(p, name, v)
    return p


def make_xsec(xs):
    x = PicXsec()
    x.n = xs.n
    x.dv_e = xs.dv_e
    x.dv_i = xs.dv_i
    keep = []
    for k, s in enumerate(xs.sigma_e):
        a = np.ascontiguousarray(s, dtype=np.float64)
        keep.append(a)
        x.sigma_e[k] = a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    for k, s in enumerate(xs.sigma_i):
        a = np.ascontiguousarray(s, dtype=np.float64)
        keep.append(a)
        x.sigma_i[k] = a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    x.exc_threshold_ev = xs.exc_threshold_ev
    x.ion_threshold_ev = xs.ion_threshold_ev
    return x, keep


def _ptr(a):
    """Device or host address of a contiguous torch tensor / numpy array."""
    if isinstance(a, torch.Tensor):
        assert a.is_contiguous()
        return ctypes.c_void_p(a.data_ptr())
    assert a.flags["C_CONTIGUOUS"]
    return ctypes.c_void_p(a.ctypes.data)


class Discharge:
    """One RF discharge on one GPU (libpic handle + its torch workspace)."""

    def __init__(self, params: dict, xs, device="cuda:0", stream=None):
        self.L = capi.load()
        self.device = torch.device(device)
        self.params = dict(params)
        self._p = make_params(params)
        self._x, self._keep = make_xsec(xs)
        nbytes = ctypes.c_uint64()
        check(self.L.pic_workspace_bytes(ctypes.byref(self._p), ctypes.byref(self._x), ctypes.byref(nbytes)),
              "pic_workspace_bytes")
        self.workspace = torch.empty(int(nbytes.value) + 256, dtype=torch.uint8, device=self.device)
        base = self.workspace.data_ptr()
        off = (-base) % 256
        # the library enqueues all of this discharge's work on this stream
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        h = ctypes.c_void_p()
        check(self.L.pic_init(ctypes.byref(self._p), ctypes.byref(self._x), ctypes.c_void_p(base + off),
                              nbytes.value, ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h)),
              "pic_init")
        self.h = h
        self.nx = int(params["n_cells"]) + 1

    def close(self):
        if getattr(self, "h", None):
            self.L.pic_free(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---- state -----------------------------------------------------------
    def set_state(self, species, x, vx, vy, vz, step=0):
        arrs = []
        for a in (x, vx, vy, vz):
            if isinstance(a, torch.Tensor):
                a = a.to(dtype=torch.float64).contiguous()
            else:
                a = np.ascontiguousarray(a, dtype=np.float64)
            arrs.append(a)
        n = int(arrs[0].shape[0])
        check(self.L.pic_set_state(self.h, species, *[_ptr(a) for a in arrs], n, int(step)), "pic_set_state")

    def count(self, species):
        n = ctypes.c_int64()
        st = ctypes.c_int64()
        s = self.L.pic_get_state(self.h, species, None, None, None, None, 0, ctypes.byref(n), ctypes.byref(st))
        if s not in (capi.PIC_OK, capi.PIC_ECAPACITY):
            check(s, "pic_get_state")
        return int(n.value)

    def get_state(self, species, to_numpy=True):
        n = self.count(species)
        out = [torch.empty(max(n, 1), dtype=torch.float64, device=self.device) for _ in range(4)]
        cnt = ctypes.c_int64()
        st = ctypes.c_int64()
        check(self.L.pic_get_state(self.h, species, *[_ptr(t) for t in out], n, ctypes.byref(cnt),
                                   ctypes.byref(st)), "pic_get_state")
        out = [t[:n] for t in out]
        if to_numpy:
            return tuple(t.cpu().numpy() for t in out)
        return tuple(out)

    def load_profile(self, species, n, dens, temp_ev, step=0):
        """Replaces the species by n particles drawn from density and
        temperature (eV) profiles at equally spaced points on [0, L]
        (libpic pic_load_profile)."""
        d = torch.as_tensor(np.asarray(dens, dtype=np.float64)).to(self.device)
        t = torch.as_tensor(np.asarray(temp_ev, dtype=np.float64)).to(self.device)
        assert d.numel() == t.numel()
        torch.cuda.current_stream(self.device).synchronize()
        check(self.L.pic_load_profile(self.h, int(species), int(n), _ptr(d), _ptr(t), d.numel(),
                                      int(step)), "pic_load_profile")

    @property
    def step_index(self):
        n = ctypes.c_int64()
        st = ctypes.c_int64()
        self.L.pic_get_state(self.h, 0, None, None, None, None, 0, ctypes.byref(n), ctypes.byref(st))
        return int(st.value)

    # ---- stepping ----------------------------------------------------------
    def step(self, n=1):
        check(self.L.pic_step(self.h, int(n)), "pic_step")

    def sync(self):
        return self.L.pic_sync(self.h)

    def set_field(self, E):
        E = np.ascontiguousarray(E, dtype=np.float64)
        assert E.size == self.nx
        check(self.L.pic_set_field(self.h, _ptr(E)), "pic_set_field")

    def get_field(self):
        nx = self.nx
        rho, phi, E = np.zeros(nx), np.zeros(nx), np.zeros(nx)
        de, di = np.zeros(nx, np.int64), np.zeros(nx, np.int64)
        check(self.L.pic_get_field(self.h, _ptr(rho), _ptr(phi), _ptr(E), _ptr(de), _ptr(di)), "pic_get_field")
        return dict(rho=rho, phi=phi, E=E, dep_e=de, dep_i=di)

    # ---- diagnostics -------------------------------------------------------
    def measure(self, on=True):
        check(self.L.pic_measure(self.h, 1 if on else 0), "pic_measure")

    def moments(self, reset=False):
        nx = self.nx
        ne, ni, em = np.zeros(nx), np.zeros(nx), np.zeros(nx)
        ep = np.zeros(int(self.params["eepf_bins"]))
        out = PicMomentsOut()
        dp = ctypes.POINTER(ctypes.c_double)
        out.n_e = ne.ctypes.data_as(dp)
        out.n_i = ni.ctypes.data_as(dp)
        out.mean_energy_e = em.ctypes.data_as(dp)
        out.eepf = ep.ctypes.data_as(dp)
        check(self.L.pic_moments(self.h, ctypes.byref(out), 1 if reset else 0), "pic_moments")
        return dict(n_e=ne, n_i=ni, mean_energy_e=em, eepf=ep, steps=int(out.steps_averaged))

    def wall_moments(self):
        """Electrode fluxes, impact energies and flux-energy distributions
        over the measured steps (libpic pic_wall_moments)."""
        nb = int(self.params["eepf_bins"])
        out = capi.PicWallOut()
        f = np.zeros((2, 2, nb))
        for k in range(2):
            for w in range(2):
                out.fedf[k][w] = f[k, w].ctypes.data_as(capi._DP)
        check(self.L.pic_wall_moments(self.h, ctypes.byref(out)), "pic_wall_moments")
        a = lambda v: np.array([[v[k][w] for w in range(2)] for k in range(2)])  # noqa: E731
        return dict(arrivals=a(out.arrivals), absorbed=a(out.absorbed), flux=a(out.flux),
                    absorbed_flux=a(out.absorbed_flux), mean_energy_ev=a(out.mean_energy_ev), fedf=f,
                    fedf_emax_ev=np.array(list(out.fedf_emax_ev)), ionizations=int(out.ionizations),
                    ionization_rate=float(out.ionization_rate), steps=int(out.steps_averaged))

    def monitors(self):
        """omega_pe dt, P_coll, Debye length, dx / lambda_D and N_D from the
        time averages (libpic pic_get_monitors)."""
        out = capi.PicMonitors()
        check(self.L.pic_get_monitors(self.h, ctypes.byref(out)), "pic_get_monitors")
        return dict(omega_pe_dt=out.omega_pe_dt, p_coll=tuple(out.p_coll), n_e_max=out.n_e_max,
                    n_e_center=out.n_e_center, mean_energy_center_ev=out.mean_energy_center_ev,
                    lambda_d_m=out.lambda_d_m, dx_over_lambda_d=out.dx_over_lambda_d, n_d=out.n_d,
                    steps=int(out.steps_averaged))

    def counters(self):
        c = np.zeros(capi.NCOUNTERS, np.int64)
        check(self.L.pic_get_counters(self.h, _ptr(c)), "pic_get_counters")
        return c

    def decisions(self, species):
        cap = max(1, int(self.params["capacity"][species]))
        buf = np.zeros(cap, np.uint8)
        n = ctypes.c_int64()
        check(self.L.pic_get_decisions(self.h, species, _ptr(buf), cap, ctypes.byref(n)), "pic_get_decisions")
        return buf[: n.value].copy()

    def set_launch(self, decide_wg_per_cu, emit_wg_per_cu):
        check(self.L.pic_set_launch(self.h, int(decide_wg_per_cu), int(emit_wg_per_cu)),
              "pic_set_launch")

    def set_pipeline(self, on=True):
        check(self.L.pic_set_pipeline(self.h, 1 if on else 0), "pic_set_pipeline")

    def set_decide_block(self, threads):
        """Decide kernels' workgroup size: 512 (default) or 256 threads."""
        check(self.L.pic_set_decide_block(self.h, int(threads)), "pic_set_decide_block")

    def tune(self, steps_per_trial=100):
        """Measures the particle kernels' launch shapes on this discharge
        (advancing it) and keeps the fastest; returns (decide, emit)
        workgroups per CU."""
        kd, ke = ctypes.c_int(), ctypes.c_int()
        check(self.L.pic_tune(self.h, int(steps_per_trial), ctypes.byref(kd), ctypes.byref(ke)),
              "pic_tune")
        return kd.value, ke.value

    def tune_pass(self, steps_per_trial=40):
        """Times the particle passes' candidate schedules and launch shapes on
        this discharge (advancing it by steps_per_trial steps per candidate)
        and keeps the fastest; returns {"trials": [...], "best": index}, each
        trial a dict of pipeline, decide_block, decide_wg_per_cu,
        emit_wg_per_cu and us_per_step."""
        from .capi import PicPassTrial

        arr = (PicPassTrial * 32)()
        n, best = ctypes.c_int(), ctypes.c_int()
        check(self.L.pic_tune_pass(self.h, int(steps_per_trial), arr, 32, ctypes.byref(n),
                                   ctypes.byref(best)), "pic_tune_pass")
        trials = [{"pipeline": bool(t.pipeline), "decide_block": t.decide_block,
                   "decide_wg_per_cu": t.decide_wg_per_cu,
                   "emit_wg_per_cu": t.emit_wg_per_cu, "us_per_step": t.us_per_step}
                  for t in arr[:min(n.value, 32)]]
        return {"trials": trials, "best": best.value}

    def timing(self, level=1):
        """0: off; 1: events around the field kernel, each species' particle
        pass and each sort; 2: also around every single particle kernel."""
        check(self.L.pic_timing(self.h, int(level)), "pic_timing")

    def get_timing(self, reset=False):
        ms = np.zeros(capi.NTIMERS)
        n = np.zeros(capi.NTIMERS, np.int64)
        check(self.L.pic_get_timing(self.h, _ptr(ms), _ptr(n), 1 if reset else 0), "pic_get_timing")
        return {name: (float(ms[i]), int(n[i])) for i, name in enumerate(capi.TIMER_NAMES)}

    def derived(self):
        d = PicDerived()
        check(self.L.pic_get_derived(self.h, ctypes.byref(d)), "pic_get_derived")
        return dict(n_x=d.n_x, n_tiles_max=d.n_tiles_max, dx=d.dx, dt=d.dt, gas_density=d.gas_density,
                    nu_max_e=d.nu_max[0], nu_max_i=d.nu_max[1], p_coll_e=d.p_coll[0], p_coll_i=d.p_coll[1])


def selftest_philox(ctr: np.ndarray, key, device="cuda:0"):
    L = capi.load()
    c = torch.as_tensor(np.ascontiguousarray(ctr, dtype=np.uint32).view(np.int32)).to(device)
    out = torch.empty_like(c)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    s = torch.cuda.current_stream(torch.device(device))
    n = c.numel() // 4
    check(L.pic_selftest_philox(_ptr(c), _ptr(k), _ptr(out), n, ctypes.c_void_p(s.cuda_stream)), "selftest_philox")
    return out.cpu().numpy().view(np.uint32).reshape(-1, 4)


def selftest_sqrt(x: np.ndarray, device="cuda:0"):
    L = capi.load()
    t = torch.as_tensor(np.ascontiguousarray(x, dtype=np.float64)).to(device)
    out = torch.empty_like(t)
    s = torch.cuda.current_stream(torch.device(device))
    check(L.pic_selftest_sqrt(_ptr(t), _ptr(out), t.numel(), ctypes.c_void_p(s.cuda_stream)), "selftest_sqrt")
    return out.cpu().numpy()


def selftest_copy(src: "torch.Tensor", dst: "torch.Tensor"):
    """Enqueues the library's plain streaming copy of src into dst (float64
    device tensors of equal, even length) on the current stream."""
    L = capi.load()
    assert src.dtype == torch.float64 and dst.dtype == torch.float64 and src.numel() == dst.numel()
    s = torch.cuda.current_stream(src.device)
    check(L.pic_selftest_copy(_ptr(src), _ptr(dst), src.numel(), ctypes.c_void_p(s.cuda_stream)),
          "selftest_copy")


def step_many(discharges, n_steps, chunk=50):
    """Advances independent discharges (each on its own stream) by n_steps
    each, interleaved so that they run concurrently; does not synchronise."""
    L = capi.load()
    arr = (ctypes.c_void_p * len(discharges))(*[d.h.value for d in discharges])
    check(L.pic_step_many(arr, len(discharges), int(n_steps), int(chunk)), "pic_step_many")


class Batch:
    """Independent discharges advanced in lockstep with one launch per
    particle pass, field solve and tail for all of them (libpic
    pic_batch_*). The discharges must share one stream; they stay usable on
    their own between batch steps and must outlive the batch."""

    def __init__(self, discharges):
        self.L = capi.load()
        self.discharges = list(discharges)
        n = len(self.discharges)
        self._arr = (ctypes.c_void_p * n)(*[d.h.value for d in self.discharges])
        nbytes = ctypes.c_uint64()
        check(self.L.pic_batch_workspace_bytes(self._arr, n, ctypes.byref(nbytes)),
              "pic_batch_workspace_bytes")
        dev = self.discharges[0].device
        self.workspace = torch.empty(int(nbytes.value) + 256, dtype=torch.uint8, device=dev)
        base = self.workspace.data_ptr()
        off = (-base) % 256
        h = ctypes.c_void_p()
        check(self.L.pic_batch_create(self._arr, n, ctypes.c_void_p(base + off), nbytes.value,
                                      ctypes.byref(h)), "pic_batch_create")
        self.h = h

    def step(self, n=1):
        check(self.L.pic_batch_step(self.h, int(n)), "pic_batch_step")

    def close(self):
        if getattr(self, "h", None):
            self.L.pic_batch_free(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Mlp:
    """The warm-start network on the GPU (libpic pic_mlp_*): n_in -> depth x
    width (GELU) -> n_out, BF16 weights with FP32 master copy, FP32
    accumulation, MSE loss, AdamW. Arrays are float32 torch tensors on the
    device, row-major [batch, features]."""

    def __init__(self, n_in, width, depth, n_out, max_batch, device="cuda:0", stream=None):
        self.L = capi.load()
        self.device = torch.device(device)
        self.dims = (int(n_in), int(width), int(depth), int(n_out))
        self.max_batch = int(max_batch)
        nbytes = ctypes.c_uint64()
        check(self.L.pic_mlp_workspace_bytes(*self.dims, self.max_batch, ctypes.byref(nbytes)),
              "pic_mlp_workspace_bytes")
        self.workspace = torch.empty(int(nbytes.value) + 256, dtype=torch.uint8, device=self.device)
        base = self.workspace.data_ptr()
        off = (-base) % 256
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        h = ctypes.c_void_p()
        check(self.L.pic_mlp_init(*self.dims, self.max_batch, ctypes.c_void_p(base + off), nbytes.value,
                                  ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h)),
              "pic_mlp_init")
        self.h = h
        n = ctypes.c_int64()
        check(self.L.pic_mlp_num_params(self.h, ctypes.byref(n)), "pic_mlp_num_params")
        self.num_params = int(n.value)

    def _f32(self, a):
        t = torch.as_tensor(a).to(device=self.device, dtype=torch.float32).contiguous()
        torch.cuda.current_stream(self.device).synchronize()
        return t

    def set_params(self, p):
        p = np.ascontiguousarray(p, dtype=np.float32)
        assert p.size == self.num_params
        check(self.L.pic_mlp_set_params(self.h, _ptr(p)), "pic_mlp_set_params")

    def get_params(self):
        p = np.zeros(self.num_params, np.float32)
        check(self.L.pic_mlp_get_params(self.h, _ptr(p)), "pic_mlp_get_params")
        return p

    def forward(self, x):
        x = self._f32(x)
        y = torch.empty((x.shape[0], self.dims[3]), dtype=torch.float32, device=self.device)
        check(self.L.pic_mlp_forward(self.h, _ptr(x), x.shape[0], _ptr(y)), "pic_mlp_forward")
        self.stream.synchronize()
        return y

    def grad(self, x, target):
        x, t = self._f32(x), self._f32(target)
        check(self.L.pic_mlp_grad(self.h, _ptr(x), _ptr(t), x.shape[0]), "pic_mlp_grad")
        g = np.zeros(self.num_params, np.float32)
        check(self.L.pic_mlp_get_grad(self.h, _ptr(g)), "pic_mlp_get_grad")
        return self.loss(), g

    def loss(self):
        v = ctypes.c_float()
        check(self.L.pic_mlp_get_loss(self.h, ctypes.byref(v)), "pic_mlp_get_loss")
        return float(v.value)

    def adam(self, lr, beta1=0.9, beta2=0.999, eps=1e-8, weight_decay=0.0):
        check(self.L.pic_mlp_adam(self.h, lr, beta1, beta2, eps, weight_decay), "pic_mlp_adam")

    def train_step(self, x, target, lr, beta1=0.9, beta2=0.999, eps=1e-8, weight_decay=0.0):
        """x, target: device float32 tensors (not copied; keep them alive until
        the stream has run the step)."""
        check(self.L.pic_mlp_train_step(self.h, _ptr(x), _ptr(target), x.shape[0], lr, beta1, beta2,
                                        eps, weight_decay), "pic_mlp_train_step")

    def close(self):
        if getattr(self, "h", None):
            self.L.pic_mlp_free(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def mlp_forward_static(dims, params, x, stream=None):
    """y = network(x) through pic_mlp_forward_static, which needs no
    workspace: dims = (n_in, width, depth, n_out); params, x: float32 device
    tensors (the parameter vector of Mlp.set_params, [batch, n_in]); returns
    [batch, n_out] after the stream has run the call."""
    L = capi.load()
    n_in, width, depth, n_out = (int(v) for v in dims)
    params = params.contiguous()
    x = x.contiguous()
    y = torch.empty((x.shape[0], n_out), dtype=torch.float32, device=x.device)
    s = stream if stream is not None else torch.cuda.current_stream(x.device)
    check(L.pic_mlp_forward_static(n_in, width, depth, n_out, _ptr(params), _ptr(x), int(x.shape[0]),
                                   _ptr(y), ctypes.c_void_p(s.cuda_stream)), "pic_mlp_forward_static")
    s.synchronize()
    return y

