"""ctypes binding of ``libimexlb.so`` (the HIP library for gfx950).

Argument marshalling only: every step of the method runs in the library's
HIP kernels.  PyTorch provides the device memory (caller-owned state and
workspace tensors) and the stream.  If the library has not been built the
import of :func:`lib` fails loudly; there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libimexlb.so")

OK, EINVAL, ENOMEM, EHIP, ENONPHYS, ESTATE = 0, -1, -2, -3, -4, -5
OUTFLOW, PERIODIC = 0, 1
F64, F32 = 0, 1


class CConfig(ctypes.Structure):
    """Mirror of ``imexlb_config``."""
    _fields_ = [("d", ctypes.c_int), ("nx", ctypes.c_int), ("ny", ctypes.c_int),
                ("lx", ctypes.c_double), ("ly", ctypes.c_double),
                ("q_phi", ctypes.c_int), ("q_chi", ctypes.c_int), ("K", ctypes.c_int),
                ("tau", ctypes.c_double), ("dt", ctypes.c_double),
                ("bc_x", ctypes.c_int), ("bc_y", ctypes.c_int), ("storage", ctypes.c_int),
                ("check_physical", ctypes.c_int)]


class CTube(ctypes.Structure):
    """Mirror of ``imexlb_tube``."""
    _fields_ = [("nx", ctypes.c_int), ("K", ctypes.c_int), ("lx", ctypes.c_double),
                ("tau", ctypes.c_double), ("dt", ctypes.c_double), ("bc", ctypes.c_int)]


BATCH_TILINGS = [(256, 0), (256, 1), (512, 0), (512, 1), (1024, 0), (1024, 1)]


@dataclass(frozen=True)
class BatchPlan:
    """One execution plan of a batch (``imexlb_batch_plan_info``)."""
    index: int
    mode: int    # 0: per-pass launches, 1: persistent launches
    tile: int
    order: int
    chunk: int
    steps: int
    bins: int


def batch_plans():
    """Every execution plan the library offers, in plan order."""
    L = lib()
    out = []
    for i in range(L.imexlb_batch_plan_count()):
        info = (ctypes.c_int * 6)()
        if L.imexlb_batch_plan_info(i, info) != OK:
            raise ImexlbError(EINVAL, f"plan {i}")
        out.append(BatchPlan(i, *list(info)))
    return out


class ImexlbError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"imexlb status {status}: {msg}")
        self.status = status


_lib = None
_vp = ctypes.c_void_p
_dp = ctypes.POINTER(ctypes.c_double)


def lib():
    """Load the library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -m paper_1909_08390_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        L.imexlb_create.argtypes = [ctypes.POINTER(CConfig), _vp, ctypes.POINTER(_vp)]
        L.imexlb_destroy.argtypes = [_vp]
        L.imexlb_destroy.restype = None
        L.imexlb_set_stream.argtypes = [_vp, _vp]
        L.imexlb_state_bytes.argtypes = [_vp]
        L.imexlb_state_bytes.restype = ctypes.c_size_t
        L.imexlb_workspace_bytes.argtypes = [_vp]
        L.imexlb_workspace_bytes.restype = ctypes.c_size_t
        L.imexlb_num_planes.argtypes = [_vp]
        L.imexlb_bind.argtypes = [_vp, _vp, _vp]
        L.imexlb_quadrature.argtypes = [_vp, _dp, _dp, _dp, _dp]
        L.imexlb_set_equilibrium.argtypes = [_vp, _vp, _vp, _vp, _vp]
        L.imexlb_set_state.argtypes = [_vp, _vp]
        L.imexlb_get_state.argtypes = [_vp, _vp]
        L.imexlb_step.argtypes = [_vp, ctypes.c_int]
        L.imexlb_step_timed.argtypes = [_vp, ctypes.c_int, _dp]
        L.imexlb_moments.argtypes = [_vp, _vp, _vp, _vp, _vp]
        L.imexlb_compute_moments.argtypes = [_vp, _vp, _vp, _vp, _vp, _vp]
        L.imexlb_advect.argtypes = [_vp, _vp, _vp]
        L.imexlb_domain_sums.argtypes = [_vp, _dp]
        L.imexlb_density_loss.argtypes = [_vp, _vp, _vp, _vp, _vp]
        L.imexlb_check_state.argtypes = [_vp]
        L.imexlb_status_string.argtypes = [ctypes.c_int]
        L.imexlb_status_string.restype = ctypes.c_char_p
        L.imexlb_last_error.argtypes = [_vp]
        L.imexlb_last_error.restype = ctypes.c_char_p
        L.imexlb_adjoint_workspace_bytes.argtypes = [_vp]
        L.imexlb_adjoint_workspace_bytes.restype = ctypes.c_size_t
        L.imexlb_adjoint_bind.argtypes = [_vp, _vp]
        L.imexlb_adjoint_step.argtypes = [_vp, _vp, _vp, _vp]
        L.imexlb_step_record_bytes.argtypes = [_vp]
        L.imexlb_step_record_bytes.restype = ctypes.c_size_t
        L.imexlb_step_recorded.argtypes = [_vp, _vp]
        L.imexlb_step_recorded_to.argtypes = [_vp, _vp, _vp]
        L.imexlb_adjoint_step_recorded.argtypes = [_vp] * 5
        L.imexlb_moments_adjoint.argtypes = [_vp] * 7
        L.imexlb_advect_adjoint.argtypes = [_vp] * 4
        L.imexlb_equilibrium_adjoint.argtypes = [_vp] * 10
        _ll = ctypes.c_longlong
        L.imexlb_batch_create.argtypes = [ctypes.POINTER(CTube), ctypes.c_int, ctypes.c_int,
                                          ctypes.c_int, ctypes.c_int, _vp, ctypes.POINTER(_vp)]
        L.imexlb_batch_destroy.argtypes = [_vp]
        L.imexlb_batch_destroy.restype = None
        L.imexlb_batch_set_stream.argtypes = [_vp, _vp]
        L.imexlb_batch_state_bytes.argtypes = [_vp]
        L.imexlb_batch_state_bytes.restype = ctypes.c_size_t
        L.imexlb_batch_workspace_bytes.argtypes = [_vp]
        L.imexlb_batch_workspace_bytes.restype = ctypes.c_size_t
        L.imexlb_batch_cells.argtypes = [_vp]
        L.imexlb_batch_cells.restype = _ll
        L.imexlb_batch_layout.argtypes = [_vp, ctypes.POINTER(_ll), ctypes.POINTER(_ll)]
        L.imexlb_batch_bind.argtypes = [_vp, _vp, _vp]
        L.imexlb_batch_set_equilibrium.argtypes = [_vp, _vp, _vp, _vp]
        L.imexlb_batch_state_changed.argtypes = [_vp]
        L.imexlb_batch_step.argtypes = [_vp, ctypes.c_int]
        L.imexlb_batch_step_timed.argtypes = [_vp, ctypes.c_int, _dp]
        L.imexlb_batch_moments.argtypes = [_vp, _vp, _vp, _vp]
        L.imexlb_batch_set_tiling.argtypes = [_vp, ctypes.c_int, ctypes.c_int]
        L.imexlb_batch_get_tiling.argtypes = [_vp, ctypes.POINTER(ctypes.c_int),
                                              ctypes.POINTER(ctypes.c_int)]
        L.imexlb_batch_tune.argtypes = [_vp, ctypes.c_int, _dp]
        L.imexlb_batch_plan_count.argtypes = []
        L.imexlb_batch_plan_info.argtypes = [ctypes.c_int, ctypes.POINTER(ctypes.c_int)]
        L.imexlb_batch_set_plan.argtypes = [_vp, ctypes.c_int]
        L.imexlb_batch_get_plan.argtypes = [_vp]
        L.imexlb_batch_last_error.argtypes = [_vp]
        L.imexlb_batch_last_error.restype = ctypes.c_char_p
        L.imexlb_copy_probe.argtypes = [_vp, _vp, ctypes.c_size_t, ctypes.c_int, _vp, _dp]
        L.imexlb_domain_sums_noalloc.argtypes = [ctypes.c_int, ctypes.c_int, _vp, _ll, _vp, _vp]
        _lib = L
    return _lib


def domain_sums_noalloc(d: int, K: int, M, stream=None):
    """Mass, momentum (x, y) and energy totals of the moment fields M, a
    contiguous FP64 device tensor (n, ux, [uy], T) of cells values each, as
    a device tensor of 4 values, by ``imexlb_domain_sums_noalloc`` (no
    allocation in the library; the output tensor is allocated here).
    Asynchronous on ``stream`` (default: torch's current stream)."""
    import torch

    nf = d + 2
    if not (M.is_cuda and M.dtype == torch.float64 and M.is_contiguous()) or M.numel() % nf:
        raise ValueError("domain_sums_noalloc: M must be a contiguous FP64 device tensor of d + 2 fields")
    out = torch.empty(4, dtype=torch.float64, device=M.device)
    st = stream if stream is not None else torch.cuda.current_stream(M.device)
    rc = lib().imexlb_domain_sums_noalloc(int(d), int(K), _vp(M.data_ptr()), M.numel() // nf,
                                          _vp(out.data_ptr()), _vp(st.cuda_stream))
    if rc != OK:
        raise ImexlbError(rc, "domain_sums_noalloc: " + lib().imexlb_status_string(rc).decode())
    return out


def copy_probe(src, dst, reps: int = 8) -> float:
    """Best rate in GB/s (read + written) of ``reps`` plain device copies of
    ``src`` into ``dst`` (contiguous CUDA tensors of one size in bytes, a
    multiple of 16) on torch's current stream: the achievable HBM rate that
    the stage passes are compared with.  ``imexlb_copy_probe``."""
    import torch

    nbytes = src.numel() * src.element_size()
    if dst.numel() * dst.element_size() != nbytes or not (src.is_contiguous() and dst.is_contiguous()):
        raise ValueError("copy_probe: src and dst must be contiguous and of the same size")
    out = ctypes.c_double(0.0)
    st = lib().imexlb_copy_probe(_vp(src.data_ptr()), _vp(dst.data_ptr()), nbytes, reps,
                                 _vp(torch.cuda.current_stream().cuda_stream), ctypes.byref(out))
    if st != OK:
        raise ImexlbError(st, lib().imexlb_status_string(st).decode())
    return out.value


@dataclass
class Config:
    """Problem definition (mirrors ``imexlb_config``)."""
    d: int
    nx: int
    ny: int = 1
    lx: float = 1.0
    ly: float = 1.0
    q_phi: int = 5
    q_chi: int = 3
    K: int = 2
    tau: float = 1e-5
    dt: float = 1e-4
    bc_x: int = OUTFLOW
    bc_y: int = OUTFLOW
    storage: int = F64
    check_physical: int = 0

    def c(self) -> CConfig:
        return CConfig(self.d, self.nx, self.ny, self.lx, self.ly,
                       self.q_phi, self.q_chi, self.K, self.tau, self.dt, self.bc_x,
                       self.bc_y, self.storage, self.check_physical)

    @property
    def planes(self) -> int:
        return self.q_phi ** self.d + self.q_chi ** self.d

    @property
    def cells(self) -> int:
        return self.nx * (self.ny if self.d == 2 else 1)

    @property
    def shape(self):
        return (self.planes, self.ny, self.nx) if self.d == 2 else (self.planes, self.nx)

    @property
    def field_shape(self):
        return (self.ny, self.nx) if self.d == 2 else (self.nx,)


def validate(cfg: Config) -> int:
    """Status of ``imexlb_create`` for cfg when it is rejected before any
    device work (EINVAL), else creates and destroys a context."""
    L = lib()
    h = _vp()
    c = cfg.c()
    st = L.imexlb_create(ctypes.byref(c), None, ctypes.byref(h))
    if st == OK:
        L.imexlb_destroy(h)
    return st


class Solver:
    """One context bound to caller-owned torch device buffers."""

    # Bytes the autograd rollout (adjoint.EquilibriumRollout) may hold in
    # recorded segments; None: 80 % of the device memory free at the time.
    rollout_memory = None

    def __init__(self, cfg: Config, device="cuda:0"):
        import torch

        self.torch = torch
        self.cfg = cfg
        self.device = torch.device(device)
        self.L = lib()
        self._h = _vp()
        with torch.cuda.device(self.device):
            stream = torch.cuda.current_stream(self.device)
            c = cfg.c()
            self._check(self.L.imexlb_create(ctypes.byref(c), _vp(stream.cuda_stream),
                                             ctypes.byref(self._h)), "create")
            self.stream = stream
            sdt = torch.float32 if cfg.storage == F32 else torch.float64
            self.state_dtype = sdt
            self.state = torch.empty(cfg.shape, dtype=sdt, device=self.device)
            assert self.state.numel() * self.state.element_size() == \
                self.L.imexlb_state_bytes(self._h)
            wb = self.L.imexlb_workspace_bytes(self._h)
            self.workspace = torch.empty(wb, dtype=torch.uint8, device=self.device)
            self._check(self.L.imexlb_bind(self._h, _vp(self.state.data_ptr()),
                                           _vp(self.workspace.data_ptr())), "bind")

    # ------------------------------------------------------------------ util
    def _check(self, st: int, what: str):
        if st != OK:
            msg = self.L.imexlb_last_error(self._h).decode() if self._h else ""
            base = self.L.imexlb_status_string(st).decode()
            raise ImexlbError(st, f"{what}: {base} {msg}".strip())

    def _dev64(self, a):
        torch = self.torch
        if a is None:
            return None
        t = torch.as_tensor(a, dtype=torch.float64, device=self.device).contiguous()
        return t.reshape(self.cfg.field_shape)

    def close(self):
        if self._h:
            self.L.imexlb_destroy(self._h)
            self._h = _vp()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ------------------------------------------------------------------- API
    @property
    def planes(self) -> int:
        return self.L.imexlb_num_planes(self._h)

    def quadrature(self):
        qp, qc = self.cfg.q_phi, self.cfg.q_chi
        pp, wp, pc, wc = (np.zeros(qp), np.zeros(qp), np.zeros(qc), np.zeros(qc))
        self._check(self.L.imexlb_quadrature(
            self._h, pp.ctypes.data_as(_dp), wp.ctypes.data_as(_dp),
            pc.ctypes.data_as(_dp), wc.ctypes.data_as(_dp)), "quadrature")
        return pp, wp, pc, wc

    def set_equilibrium(self, n, ux, uy, T):
        n, ux, T = self._dev64(n), self._dev64(ux), self._dev64(T)
        uy = self._dev64(uy) if self.cfg.d == 2 else None
        self._keep = (n, ux, uy, T)  # alive until the stream has used them
        self._check(self.L.imexlb_set_equilibrium(
            self._h, _vp(n.data_ptr()), _vp(ux.data_ptr()),
            _vp(uy.data_ptr()) if uy is not None else None, _vp(T.data_ptr())), "set_equilibrium")

    def bind_state(self, F):
        """Bind the tensor F (state shape and dtype, contiguous) as the state
        buffer, keeping the workspace (``imexlb_bind``), and take its moments
        (``imexlb_set_state`` without a copy).  Out-of-place steps then read
        F without modifying it."""
        assert F.dtype == self.state_dtype and tuple(F.shape) == tuple(self.cfg.shape)
        assert F.is_contiguous() and F.device == self.device
        self._check(self.L.imexlb_bind(self._h, _vp(F.data_ptr()), _vp(self.workspace.data_ptr())), "bind")
        self.state = F
        self._check(self.L.imexlb_set_state(self._h, _vp(F.data_ptr())), "set_state")

    def set_state(self, F):
        F = self.torch.as_tensor(F, dtype=self.state_dtype, device=self.device).contiguous()
        assert tuple(F.shape) == tuple(self.cfg.shape)
        self._keep = F
        self._check(self.L.imexlb_set_state(self._h, _vp(F.data_ptr())), "set_state")

    def step(self, nsteps: int = 1):
        self._check(self.L.imexlb_step(self._h, int(nsteps)), "step")

    def side_stream(self):
        """A second stream of default priority, created on first use and kept
        for the solver's life (the caching allocator keeps each stream's freed
        blocks for that stream, so one kept stream reuses them)."""
        if getattr(self, "_side", None) is None:
            self._side = self.torch.cuda.Stream(device=self.device)
        return self._side

    def set_stream(self, stream):
        """Run the following calls on ``stream`` (a torch.cuda.Stream of
        default priority); ``imexlb_set_stream``."""
        self._check(self.L.imexlb_set_stream(self._h, _vp(stream.cuda_stream)), "set_stream")
        self.stream = stream

    def step_timed(self, nsteps: int):
        """Step and return the summed per-pass milliseconds (stage 3, 4, 5),
        timed with HIP events on the library's stream."""
        ms = np.zeros(3)
        self._check(self.L.imexlb_step_timed(self._h, int(nsteps), ms.ctypes.data_as(_dp)),
                    "step_timed")
        return ms

    def moments(self):
        """(n, ux, uy, T) device tensors of the current state (uy zero in 1D)."""
        torch = self.torch
        out = [torch.zeros(self.cfg.field_shape, dtype=torch.float64, device=self.device)
               for _ in range(4)]
        self._check(self.L.imexlb_moments(self._h, *[_vp(t.data_ptr()) for t in out]), "moments")
        return tuple(out)

    def compute_moments(self, F):
        torch = self.torch
        F = torch.as_tensor(F, dtype=self.state_dtype, device=self.device).contiguous()
        out = [torch.zeros(self.cfg.field_shape, dtype=torch.float64, device=self.device)
               for _ in range(4)]
        self._check(self.L.imexlb_compute_moments(self._h, _vp(F.data_ptr()),
                                                  *[_vp(t.data_ptr()) for t in out]),
                    "compute_moments")
        return tuple(out)

    def advect(self, F):
        """FP64 (p . grad) F of a plane-set (the MP-9 operator alone)."""
        torch = self.torch
        F = torch.as_tensor(F, dtype=self.state_dtype, device=self.device).contiguous()
        VF = torch.empty(self.cfg.shape, dtype=torch.float64, device=self.device)
        self._check(self.L.imexlb_advect(self._h, _vp(F.data_ptr()), _vp(VF.data_ptr())), "advect")
        return VF

    def domain_sums(self) -> np.ndarray:
        out = np.zeros(4)
        self._check(self.L.imexlb_domain_sums(self._h, out.ctypes.data_as(_dp)), "domain_sums")
        return out

    def density_loss(self, target, n=None, grad: bool = False):
        """(loss, grad): 1/2 sum (n - target)^2 as a 0-d FP64 device tensor
        and, when ``grad``, the field n - target; n defaults to the density
        of the current state.  ``imexlb_density_loss``."""
        torch = self.torch
        target = self._dev64(target)
        n = self._dev64(n) if n is not None else None
        loss = torch.empty((), dtype=torch.float64, device=self.device)
        g = torch.empty(self.cfg.field_shape, dtype=torch.float64, device=self.device) if grad else None
        self._keep = (n, target)
        self._check(self.L.imexlb_density_loss(
            self._h, _vp(n.data_ptr()) if n is not None else None, _vp(target.data_ptr()),
            _vp(loss.data_ptr()), _vp(g.data_ptr()) if g is not None else None), "density_loss")
        return loss, g

    def check_state(self) -> int:
        return self.L.imexlb_check_state(self._h)

    # --------------------------------------------------------------- adjoint
    def adjoint_bind(self):
        """Allocate and bind the adjoint workspace (once)."""
        if getattr(self, "adj_workspace", None) is None:
            torch = self.torch
            nb = self.L.imexlb_adjoint_workspace_bytes(self._h)
            self.adj_workspace = torch.empty(nb, dtype=torch.uint8, device=self.device)
            self._check(self.L.imexlb_adjoint_bind(self._h, _vp(self.adj_workspace.data_ptr())),
                        "adjoint_bind")

    def _dev_planes64(self, x):
        t = self.torch.as_tensor(x, dtype=self.torch.float64, device=self.device).contiguous()
        assert tuple(t.shape) == tuple(self.cfg.shape)
        return t

    def new_record(self):
        """A device buffer for one recorded step (imexlb_step_record_bytes)."""
        nb = self.L.imexlb_step_record_bytes(self._h)
        return self.torch.empty(nb, dtype=self.torch.uint8, device=self.device)

    def step_recorded(self, record, out=None):
        """One step that also leaves its stage sources and moments in record
        (a buffer from new_record) for adjoint_step.  With ``out`` (a tensor
        like ``state``) the step is out of place (``imexlb_step_recorded_to``):
        F^{n+1} goes to ``out``, which becomes ``self.state``, and the tensor
        that was ``self.state`` keeps F^n."""
        assert record.numel() >= self.L.imexlb_step_record_bytes(self._h) and record.data_ptr() % 256 == 0
        if out is None:
            self._check(self.L.imexlb_step_recorded(self._h, _vp(record.data_ptr())), "step_recorded")
            return
        assert out.dtype == self.state_dtype and tuple(out.shape) == tuple(self.cfg.shape)
        assert out.is_contiguous() and out.device == self.device
        self._check(self.L.imexlb_step_recorded_to(self._h, _vp(record.data_ptr()), _vp(out.data_ptr())),
                    "step_recorded_to")
        self.state = out

    def adjoint_step(self, Fn, lam1, record=None):
        """(dF^{n+1}/dF^n)^T lam1 for the step taken from state Fn; with the
        record that step_recorded left for that step, the forward stage
        sources are read instead of recomputed."""
        self.adjoint_bind()
        Fn = self.torch.as_tensor(Fn, dtype=self.state_dtype, device=self.device).contiguous()
        lam1 = self._dev_planes64(lam1)
        lam0 = self.torch.empty_like(lam1)
        if record is None:
            st = self.L.imexlb_adjoint_step(self._h, _vp(Fn.data_ptr()), _vp(lam1.data_ptr()),
                                            _vp(lam0.data_ptr()))
        else:
            assert record.numel() >= self.L.imexlb_step_record_bytes(self._h)
            st = self.L.imexlb_adjoint_step_recorded(self._h, _vp(Fn.data_ptr()), _vp(record.data_ptr()),
                                                     _vp(lam1.data_ptr()), _vp(lam0.data_ptr()))
        self._check(st, "adjoint_step")
        return lam0

    def advect_adjoint(self, F, dA):
        """V^T dA at the FP64 plane-set F (transpose of advect)."""
        F = self._dev_planes64(F)
        dA = self._dev_planes64(dA)
        dF = self.torch.empty_like(dA)
        self._check(self.L.imexlb_advect_adjoint(self._h, _vp(F.data_ptr()), _vp(dA.data_ptr()),
                                                 _vp(dF.data_ptr())), "advect_adjoint")
        return dF

    def moments_adjoint(self, F, dn, dux, duy, dT):
        self.adjoint_bind()
        torch = self.torch
        F = torch.as_tensor(F, dtype=self.state_dtype, device=self.device).contiguous()
        f = [self._dev64(x if x is not None else np.zeros(self.cfg.field_shape))
             for x in (dn, dux, duy, dT)]
        lam = torch.empty(self.cfg.shape, dtype=torch.float64, device=self.device)
        self._check(self.L.imexlb_moments_adjoint(self._h, _vp(F.data_ptr()),
                                                  *[_vp(t.data_ptr()) for t in f],
                                                  _vp(lam.data_ptr())), "moments_adjoint")
        return lam

    def equilibrium_adjoint(self, n, ux, uy, T, lam):
        """Gradients (dn, dux, duy, dT) of <lam, E(n, u, T)>."""
        self.adjoint_bind()
        torch = self.torch
        f = [self._dev64(x if x is not None else np.zeros(self.cfg.field_shape)) for x in (n, ux, uy, T)]
        lam = self._dev_planes64(lam)
        out = [torch.empty(self.cfg.field_shape, dtype=torch.float64, device=self.device) for _ in range(4)]
        self._check(self.L.imexlb_equilibrium_adjoint(self._h, *[_vp(t.data_ptr()) for t in f],
                                                      _vp(lam.data_ptr()),
                                                      *[_vp(t.data_ptr()) for t in out]),
                    "equilibrium_adjoint")
        return tuple(out)


@dataclass
class TubeSpec:
    """One tube of a batch (mirrors ``imexlb_tube``)."""
    nx: int
    K: int = 2
    lx: float = 1.0
    tau: float = 1e-5
    dt: float = 1e-4
    bc: int = OUTFLOW

    def c(self) -> CTube:
        return CTube(self.nx, self.K, self.lx, self.tau, self.dt, self.bc)


def batch_validate(tubes, q_phi=8, q_chi=8, storage=F32) -> int:
    """Status of ``imexlb_batch_create`` (EINVAL before any device work)."""
    L = lib()
    arr = (CTube * max(len(tubes), 1))(*[t.c() for t in tubes])
    h = _vp()
    st = L.imexlb_batch_create(arr, len(tubes), q_phi, q_chi, storage, None, ctypes.byref(h))
    if st == OK:
        L.imexlb_batch_destroy(h)
    return st


class Batch:
    """Many 1D tubes of uneven size advanced together (one launch per pass),
    bound to caller-owned torch device buffers."""

    def __init__(self, tubes, q_phi=8, q_chi=8, storage=F32, device="cuda:0"):
        import torch

        self.torch = torch
        self.tubes = list(tubes)
        self.q_phi, self.q_chi, self.storage = q_phi, q_chi, storage
        self.planes = q_phi + q_chi
        self.device = torch.device(device)
        self.L = lib()
        self._h = _vp()
        arr = (CTube * len(self.tubes))(*[t.c() for t in self.tubes])
        with torch.cuda.device(self.device):
            self.stream = torch.cuda.current_stream(self.device)
            self._check(self.L.imexlb_batch_create(arr, len(self.tubes), q_phi, q_chi, storage,
                                                   _vp(self.stream.cuda_stream),
                                                   ctypes.byref(self._h)), "batch_create")
            self.state_dtype = torch.float32 if storage == F32 else torch.float64
            esz = 4 if storage == F32 else 8
            sb = self.L.imexlb_batch_state_bytes(self._h)
            # zeroed so that the padding between tubes holds defined values
            self.state = torch.zeros(sb // esz, dtype=self.state_dtype, device=self.device)
            self.workspace = torch.empty(self.L.imexlb_batch_workspace_bytes(self._h),
                                         dtype=torch.uint8, device=self.device)
            self._check(self.L.imexlb_batch_bind(self._h, _vp(self.state.data_ptr()),
                                                 _vp(self.workspace.data_ptr())), "batch_bind")
        self.cells = self.L.imexlb_batch_cells(self._h)
        so = (ctypes.c_longlong * len(self.tubes))()
        co = (ctypes.c_longlong * len(self.tubes))()
        self._check(self.L.imexlb_batch_layout(self._h, so, co), "batch_layout")
        self.state_offset = list(so)
        self.cell_offset = list(co)

    def _check(self, st: int, what: str):
        if st != OK:
            msg = self.L.imexlb_batch_last_error(self._h).decode() if self._h else ""
            base = self.L.imexlb_status_string(st).decode()
            raise ImexlbError(st, f"{what}: {base} {msg}".strip())

    def close(self):
        if self._h:
            self.L.imexlb_batch_destroy(self._h)
            self._h = _vp()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def tube_state(self, i):
        """View of tube i's plane-set, shape (planes, nx)."""
        o, nx = self.state_offset[i], self.tubes[i].nx
        return self.state[o:o + self.planes * nx].view(self.planes, nx)

    def concat(self, per_tube):
        """One FP64 device array over all cells from per-tube arrays."""
        torch = self.torch
        return torch.cat([torch.as_tensor(a, dtype=torch.float64).reshape(-1)
                          for a in per_tube]).to(self.device).contiguous()

    def split(self, field):
        return [field[c:c + t.nx] for c, t in zip(self.cell_offset, self.tubes)]

    def set_equilibrium(self, n, u, T):
        """n, u, T: per-tube lists of arrays, or arrays over all cells."""
        f = [self.concat(x) if isinstance(x, (list, tuple)) else
             self.torch.as_tensor(x, dtype=self.torch.float64, device=self.device).contiguous()
             for x in (n, u, T)]
        self._keep = f
        self._check(self.L.imexlb_batch_set_equilibrium(self._h, *[_vp(t.data_ptr()) for t in f]),
                    "batch_set_equilibrium")

    def state_changed(self):
        self._check(self.L.imexlb_batch_state_changed(self._h), "batch_state_changed")

    def step(self, nsteps: int = 1):
        self._check(self.L.imexlb_batch_step(self._h, int(nsteps)), "batch_step")

    def step_timed(self, nsteps: int):
        ms = np.zeros(3)
        self._check(self.L.imexlb_batch_step_timed(self._h, int(nsteps), ms.ctypes.data_as(_dp)),
                    "batch_step_timed")
        return ms

    def moments(self):
        """(n, u, T) device tensors over all cells."""
        torch = self.torch
        out = [torch.zeros(self.cells, dtype=torch.float64, device=self.device) for _ in range(3)]
        self._check(self.L.imexlb_batch_moments(self._h, *[_vp(t.data_ptr()) for t in out]),
                    "batch_moments")
        return tuple(out)

    def set_tiling(self, tile: int, order: int = 0):
        self._check(self.L.imexlb_batch_set_tiling(self._h, int(tile), int(order)), "batch_set_tiling")

    def tiling(self):
        t, o = ctypes.c_int(), ctypes.c_int()
        self._check(self.L.imexlb_batch_get_tiling(self._h, ctypes.byref(t), ctypes.byref(o)),
                    "batch_get_tiling")
        return t.value, o.value

    def set_plan(self, plan):
        """Execution plan by index or BatchPlan."""
        idx = plan.index if isinstance(plan, BatchPlan) else int(plan)
        self._check(self.L.imexlb_batch_set_plan(self._h, idx), "batch_set_plan")

    def plan(self) -> BatchPlan:
        return batch_plans()[self.L.imexlb_batch_get_plan(self._h)]

    def tune(self, nsteps: int = 5):
        """Autotune over every plan; returns {BatchPlan: ms per step} and
        leaves the fastest plan set."""
        plans = batch_plans()
        ms = np.zeros(len(plans))
        self._check(self.L.imexlb_batch_tune(self._h, int(nsteps), ms.ctypes.data_as(_dp)),
                    "batch_tune")
        return dict(zip(plans, ms.tolist()))
