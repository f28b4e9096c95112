"""Python-side handle of one libpm context: torch owns the device workspace and
the stream; every call forwards to the C ABI (include/pm.h)."""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass, fields

import torch

from . import _lib


@dataclass
class Config:
    """Mirror of pm_config (include/pm.h); defaults are the paper's PM
    defaults where it gives one (tab. default_parameters)."""
    n_p: int = 32
    n_g: int = 64
    box: float = 100.0
    omega_m: float = 0.31
    h: float = 0.68
    n_s: float = 0.965
    sigma8: float = 0.81
    spectrum: str = "bbks"        # "bbks" | "powerlaw"
    pl_rms_cells: float = 0.2
    a_start: float = 0.02
    a_end: float = 1.0
    n_steps: int = 10
    force: str = "pm"             # "pm" | "nufft"
    mak: int = 2                  # 2 CIC, 3 TSC
    deconvolve: bool = False
    grad_order: int = 4
    lap_order: int = 0
    es_width: int = 6
    es_beta: float = 13.8
    batch: int = 1
    lpt_order: int = 1            # 1 Zel'dovich, 2 second-order LPT initial state
    stepper: str = "bullfrog"     # "bullfrog" | "fastpm" | "leapfrog" (canonical momentum)
    time_var: str = "D"           # step spacing uniform in "D" | "a" | "lna" | "superconft"
    antialias: int = 0            # 1: interlaced grids for the PM force

    def to_c(self):
        c = _lib.pm_config()
        for f in fields(self):
            v = getattr(self, f.name)
            if f.name == "spectrum":
                v = _lib.PM_SPEC_BBKS if v == "bbks" else _lib.PM_SPEC_POWERLAW
            elif f.name == "force":
                v = _lib.PM_FORCE_PM if v == "pm" else _lib.PM_FORCE_NUFFT
            elif f.name == "stepper":
                v = {"bullfrog": 0, "fastpm": 1, "leapfrog": 2}[v]
            elif f.name == "time_var":
                v = {"D": 0, "a": 1, "lna": 2, "superconft": 3}[v]
            elif isinstance(v, bool):
                v = int(v)
            setattr(c, f.name, v)
        return c

    @property
    def N(self):
        return self.n_p ** 3

    @property
    def M(self):
        return self.n_g ** 3


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else None


class PMSim:
    """One context of B same-shape slots bound to a torch-owned workspace."""

    def __init__(self, cfg: Config, with_adjoint=False, device="cuda"):
        self.lib = _lib.load()
        self.cfg = cfg
        self.device = torch.device(device)
        self.state_token = 0      # bumped by every call that changes the particle state
        ctx = C.c_void_p()
        ccfg = cfg.to_c()
        _lib.check(self.lib.pm_create(C.byref(ccfg), C.byref(ctx)), None, "pm_create")
        self.ctx = ctx
        self.with_adjoint = bool(with_adjoint)
        nbytes = int(self.lib.pm_workspace_bytes(ctx, int(self.with_adjoint)))
        self.workspace_bytes = nbytes
        self._ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        off = (-self._ws.data_ptr()) % 256
        self.stream = torch.cuda.current_stream(self.device)
        _lib.check(self.lib.pm_bind(ctx, C.c_void_p(self._ws.data_ptr() + off), nbytes,
                                    int(self.with_adjoint), C.c_void_p(self.stream.cuda_stream)),
                   ctx, "pm_bind")

    def __del__(self):
        ctx = getattr(self, "ctx", None)
        if ctx:
            self.lib.pm_destroy(ctx)
            self.ctx = None

    # --------------------------------------------------------------- calls
    _STATE_CALLS = frozenset({"pm_init_ics", "pm_step", "pm_run", "pm_adjoint", "pm_adjoint_full", "pm_set_state",
                              "pm_deposit",
                              "pm_force", "pm_force_vjp", "pm_set_active", "pm_step_device", "pm_jvp"})

    def _call(self, name, *args):
        if name in self._STATE_CALLS:
            self.state_token += 1
        _lib.check(getattr(self.lib, name)(self.ctx, *args), self.ctx, name)

    def _new(self, *shape, dtype=torch.float32):
        return torch.empty(*shape, dtype=dtype, device=self.device)

    def set_slot_params(self, n_steps=None, sigma8=None):
        B = self.cfg.batch
        ns = (C.c_int32 * B)(*n_steps) if n_steps is not None else None
        sg = (C.c_double * B)(*sigma8) if sigma8 is not None else None
        self._call("pm_set_slot_params", ns, sg)

    def init_ics(self, seeds=None, w=None, return_w=False):
        B, N = self.cfg.batch, self.cfg.N
        sd = (C.c_uint64 * B)(*[int(s) for s in seeds]) if seeds is not None else None
        if w is not None:
            w = w.to(self.device, torch.float32).contiguous().reshape(B, N)
        w_out = self._new(B, N) if return_w else None
        self._call("pm_init_ics", sd, _ptr(w), _ptr(w_out))
        return w_out

    def step(self, step_index):
        B = self.cfg.batch
        self._call("pm_step", (C.c_int32 * B)(*step_index))

    def run(self):
        self._call("pm_run")

    def set_step_index(self, step_index):
        """Device step index per slot: k >= 0 next step, -1 idle, -2 keep."""
        B = self.cfg.batch
        self._call("pm_set_step_index", (C.c_int32 * B)(*[int(k) for k in step_index]))

    def step_device(self):
        """Advance every slot with a device step index >= 0 by one step."""
        self._call("pm_step_device")

    def get_step_index(self):
        B = self.cfg.batch
        out = (C.c_int32 * B)()
        self._call("pm_get_step_index", out)
        return list(out)

    def adjoint(self, dL_ddelta, temporal=False):
        """(dL/dw [B, N], dL/dsigma8 [B]); with temporal, also the adjoints of
        every step's (tau1, tau2, alpha, beta) [B, n_steps, 4]."""
        B = self.cfg.batch
        g = dL_ddelta.to(self.device, torch.float32).contiguous().reshape(B, self.cfg.M)
        dw = self._new(B, self.cfg.N)
        ds = self._new(B, dtype=torch.float64)
        if not temporal:
            self._call("pm_adjoint", _ptr(g), _ptr(dw), _ptr(ds))
            return dw, ds
        dt = self._new(B, self.cfg.n_steps, 4, dtype=torch.float64)
        self._call("pm_adjoint_full", _ptr(g), _ptr(dw), _ptr(ds), _ptr(dt))
        return dw, ds, dt

    def power_spectrum(self, n_bins, deconvolve=True):
        B = self.cfg.batch
        k = self._new(B, n_bins, dtype=torch.float64)
        p = self._new(B, n_bins, dtype=torch.float64)
        n = self._new(B, n_bins, dtype=torch.int64)
        self._call("pm_power_spectrum", int(n_bins), int(bool(deconvolve)), _ptr(k), _ptr(p), _ptr(n))
        return k, p, n

    def jvp(self, w_dot, sigma8_dot=None):
        """Forward-mode tangent of the final CIC contrast [B, M] along
        (w_dot [B, N], sigma8_dot [B]); reruns the forward from the white
        noise of init_ics and leaves the context at its final state."""
        B = self.cfg.batch
        wd = w_dot.to(self.device, torch.float32).contiguous().reshape(B, self.cfg.N)
        sd = (C.c_double * B)(*[float(x) for x in sigma8_dot]) if sigma8_dot is not None else None
        dd = self._new(B, self.cfg.M)
        self._call("pm_jvp", _ptr(wd), sd, _ptr(dd))
        return dd

    def get_tangent(self):
        """(Xdot, Vdot) [B, 3, N] of the final state after jvp."""
        B, N = self.cfg.batch, self.cfg.N
        x, v = self._new(B, 3, N), self._new(B, 3, N)
        self._call("pm_get_tangent", _ptr(x), _ptr(v))
        return x, v

    def power_spectrum_jvp(self, delta_dot, n_bins, deconvolve=True):
        """(k, P, P_dot, counts) of the current final state, P_dot the
        tangent of P when the contrast moves along delta_dot [B, M]."""
        B = self.cfg.batch
        dd = delta_dot.to(self.device, torch.float32).contiguous().reshape(B, self.cfg.M)
        k = self._new(B, n_bins, dtype=torch.float64)
        p = self._new(B, n_bins, dtype=torch.float64)
        pd = self._new(B, n_bins, dtype=torch.float64)
        n = self._new(B, n_bins, dtype=torch.int64)
        self._call("pm_power_spectrum_jvp", _ptr(dd), int(n_bins), int(bool(deconvolve)), _ptr(k), _ptr(p),
                   _ptr(pd), _ptr(n))
        return k, p, pd, n

    def density(self, fixed=False):
        B = self.cfg.batch
        d = self._new(B, self.cfg.M)
        f = self._new(B, self.cfg.M, dtype=torch.int64) if fixed else None
        self._call("pm_density", _ptr(d), _ptr(f))
        return (d, f) if fixed else d

    def get_state(self):
        B, N = self.cfg.batch, self.cfg.N
        x, v = self._new(B, 3, N), self._new(B, 3, N)
        self._call("pm_get_state", _ptr(x), _ptr(v))
        return x, v

    def set_state(self, disp, vel):
        B, N = self.cfg.batch, self.cfg.N
        x = disp.to(self.device, torch.float32).contiguous().reshape(B, 3, N)
        v = vel.to(self.device, torch.float32).contiguous().reshape(B, 3, N)
        self._call("pm_set_state", _ptr(x), _ptr(v))

    def deposit(self, disp, mak):
        B, N = self.cfg.batch, self.cfg.N
        x = disp.to(self.device, torch.float32).contiguous().reshape(B, 3, N)
        m = self._new(B, self.cfg.M, dtype=torch.int64)
        self._call("pm_deposit", _ptr(x), int(mak), _ptr(m))
        return m

    def force(self, disp, s):
        B, N = self.cfg.batch, self.cfg.N
        x = disp.to(self.device, torch.float32).contiguous().reshape(B, 3, N)
        a = self._new(B, 3, N)
        self._call("pm_force", _ptr(x), float(s), _ptr(a))
        return a

    def force_vjp(self, disp, s, u, parts=3):
        """J_A(disp)^T u of the force (parts: 1 direct, 2 through the mesh, 3 both)."""
        B, N = self.cfg.batch, self.cfg.N
        x = disp.to(self.device, torch.float32).contiguous().reshape(B, 3, N)
        uu = u.to(self.device, torch.float32).contiguous().reshape(B, 3, N)
        out = self._new(B, 3, N)
        self._call("pm_force_vjp", _ptr(x), float(s), _ptr(uu), int(parts), _ptr(out))
        return out

    def fft(self, x, inverse=False):
        B, n = self.cfg.batch, self.cfg.n_g
        if not inverse:
            xin = x.to(self.device, torch.float32).contiguous().reshape(B, n, n, n)
            out = self._new(B, n, n, n // 2 + 1, dtype=torch.complex64)
        else:
            xin = x.to(self.device, torch.complex64).contiguous().reshape(B, n, n, n // 2 + 1)
            out = self._new(B, n, n, n)
        self._call("pm_fft", _ptr(xin), _ptr(out), int(bool(inverse)))
        return out

    def synchronize(self):
        self.stream.synchronize()

    def set_active(self, slots=None):
        """Restrict whole-context calls to the given slot indices (None: all)."""
        B = self.cfg.batch
        mask = (1 << B) - 1 if slots is None else sum(1 << int(b) for b in slots)
        self._call("pm_set_active", C.c_uint64(mask))

    def profile(self, on=True):
        self._call("pm_profile", int(bool(on)))

    def use_graphs(self, on=True):
        """Replay run() from a captured HIP graph (default) or launch eagerly."""
        self._call("pm_use_graphs", int(bool(on)))

    def kernel_times(self):
        """{class: (total ms, launches)} since the previous call (synchronises)."""
        K = len(_lib.KERNEL_CLASSES)
        ms = (C.c_double * K)()
        n = (C.c_int64 * K)()
        self._call("pm_kernel_times", C.cast(ms, C.c_void_p), C.cast(n, C.c_void_p))
        return {name: (ms[i], n[i]) for i, name in enumerate(_lib.KERNEL_CLASSES)}


class PMFunction(torch.autograd.Function):
    """delta = F(w, sigma8) behind torch autograd (Sec. "Automatic
    differentiation", Sec. "Adjoint method").

    forward(w [B, N], sigma8 [B], sim) sets each slot's sigma8, runs the
    initial conditions and the BullFrog steps on the GPU and returns the final
    CIC density contrast [B, n_g^3]; it saves no trajectory, only the context.
    backward(delta_bar) runs pm_adjoint, which integrates the primal state and
    the cotangents back to the initial conditions (memory independent of the
    number of steps), and returns (w_bar, sigma8_bar, None).  The context must
    still hold this forward's final state: any later call that changes it
    (another forward, a step, set_state, a test hook) makes backward raise."""

    @staticmethod
    def forward(ctx, w, sigma8, sim):
        B, N = sim.cfg.batch, sim.cfg.N
        if w.numel() != B * N:
            raise ValueError(f"w must hold {B} x {N} values")
        s8 = torch.as_tensor(sigma8, dtype=torch.float64).detach().reshape(-1).cpu()
        if s8.numel() != B:
            raise ValueError(f"sigma8 must hold {B} values")
        sim.set_slot_params(sigma8=[float(v) for v in s8])
        sim.init_ics(w=w.detach())
        sim.run()
        delta = sim.density()
        ctx.sim = sim
        ctx.token = sim.state_token
        ctx.w_shape, ctx.w_dtype = w.shape, w.dtype
        st = torch.as_tensor(sigma8)
        ctx.s_shape, ctx.s_dtype, ctx.s_device = st.shape, st.dtype, st.device
        return delta

    @staticmethod
    def backward(ctx, g):
        sim = ctx.sim
        if sim.state_token != ctx.token:
            raise RuntimeError("PMFunction.backward: the context no longer holds this forward's final state "
                               "(it was run or modified after the forward)")
        dw, ds = sim.adjoint(g)
        ctx.sim = None
        return (dw.reshape(ctx.w_shape).to(ctx.w_dtype),
                ds.reshape(ctx.s_shape).to(device=ctx.s_device, dtype=ctx.s_dtype), None)


def simulate(w, sigma8, sim):
    """Differentiable forward model: final CIC density contrast of the white
    noise w and sigma8 (PMFunction.apply)."""
    return PMFunction.apply(w, sigma8, sim)


def power_spectrum_of_mesh_noalloc(mesh, n_particles, box, n_bins, deconvolve=True):
    """P(k) of an int64 fixed-point CIC mass mesh (n^3 on the GPU, n <= 128)
    through pm_power_spectrum_mesh_noalloc, which allocates nothing: the
    outputs are allocated here by torch; returns (k_mean, pk, n_modes)."""
    assert mesh.is_cuda and mesh.dtype == torch.int64 and mesh.is_contiguous()
    n = round(mesh.numel() ** (1.0 / 3.0))
    assert n ** 3 == mesh.numel()
    k = torch.empty(n_bins, dtype=torch.float64, device=mesh.device)
    p = torch.empty_like(k)
    c = torch.empty(n_bins, dtype=torch.int64, device=mesh.device)
    st = _lib.load().pm_power_spectrum_mesh_noalloc(
        _ptr(mesh), n, int(n_particles), float(box), int(n_bins), int(bool(deconvolve)), _ptr(k), _ptr(p), _ptr(c),
        C.c_void_p(torch.cuda.current_stream(mesh.device).cuda_stream))
    _lib.check(st, None, "pm_power_spectrum_mesh_noalloc")
    return k, p, c
