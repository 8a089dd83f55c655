"""Python binding of libfmm.so (include/fmm.h): argument marshalling only.

Every function here forwards to the C ABI function of the same name; device
buffers are torch tensors on a HIP device, streams are torch streams.  No
arithmetic of the method runs in Python, and there is no fallback: if the
library is missing or fails to load, ``load()`` raises.

``FMM`` is a small convenience owner of one workspace and one plan.
"""
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfmm.so")

FMM_ABI_VERSION = 2
FMM_P_MAX = 12
FMM_DEPTH_MAX = 9
FMM_PREC_FP64, FMM_PREC_MIXED = 0, 1
FMM_M2L_AUTO, FMM_M2L_F64, FMM_M2L_F32, FMM_M2L_BF16X2, FMM_M2L_BF16X3, FMM_M2L_F16X2 = 0, 1, 2, 3, 4, 5
STATUS_NAMES = {0: "FMM_OK", 1: "FMM_E_INVALID_ARG", 2: "FMM_E_WORKSPACE", 3: "FMM_E_OUT_OF_CUBE",
                4: "FMM_E_NONFINITE", 5: "FMM_E_COINCIDENT", 6: "FMM_E_UNSUPPORTED",
                7: "FMM_E_DEVICE"}
PHASES = ["tree", "operators", "p2m", "m2m", "m2l", "l2l", "l2p", "p2p", "energy", "split"]

# every symbol include/fmm.h declares
EXPORTS = ["fmm_config_default", "fmm_workspace_size", "fmm_plan", "fmm_evaluate", "fmm_backward",
           "fmm_check", "fmm_destroy", "fmm_status_string", "fmm_plan_leaves", "fmm_plan_cube",
           "fmm_hilbert_index", "fmm_profile_enable", "fmm_profile_read", "fmm_plan_work", "fmm_plan_tree_stats",
           "fmm_evaluate_static", "fmm_replan", "fmm_plan_set_schedule"]
FMM_SCHED_P2P_PERSISTENT, FMM_SCHED_M2L_SPLIT, FMM_SCHED_M2L_PERSISTENT, FMM_SCHED_P2P_TILE = 0, 1, 2, 3
FMM_STATIC_SCRATCH_BYTES = 128 << 20


class fmm_config(ctypes.Structure):
    _fields_ = [("abi_version", ctypes.c_uint32), ("p", ctypes.c_int32), ("depth", ctypes.c_int32),
                ("leaf_max", ctypes.c_int32), ("ws", ctypes.c_int32),
                ("precision", ctypes.c_int32), ("m2l_kind", ctypes.c_int32),
                ("root_lo", ctypes.c_double * 3), ("root_side", ctypes.c_double),
                ("batch_level", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class FMMError(RuntimeError):
    def __init__(self, status, what=""):
        self.status = status
        super().__init__(f"{what}: {STATUS_NAMES.get(status, status)}")


_LIB = None


def load(path=LIB_PATH):
    """Load libfmm.so (raises OSError when it is missing or unloadable).

    torch is imported first so that the library binds to the HIP runtime torch
    already mapped (torch ships its own libamdhip64 with the same soname);
    loading the library first would map a second runtime, in which torch's
    device pointers and streams are not valid."""
    global _LIB
    if _LIB is not None and path == LIB_PATH:
        return _LIB
    import torch  # noqa: F401  (see above)
    if not os.path.exists(path):
        raise OSError(f"{path} is not built; run paper_2209_13121_amd/build.py")
    lib = ctypes.CDLL(path)
    vp, i64, i32, dp = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.POINTER(ctypes.c_double)
    cfgp = ctypes.POINTER(fmm_config)
    lib.fmm_config_default.argtypes = [cfgp]
    lib.fmm_config_default.restype = None
    lib.fmm_workspace_size.argtypes = [cfgp, i64, ctypes.POINTER(ctypes.c_size_t)]
    lib.fmm_plan.argtypes = [cfgp, i64, vp, vp, ctypes.c_size_t, vp, ctypes.POINTER(vp)]
    lib.fmm_evaluate.argtypes = [vp, vp, vp, vp, vp, vp]
    lib.fmm_backward.argtypes = [vp, vp, vp, vp, vp]
    lib.fmm_check.argtypes = [vp]
    lib.fmm_destroy.argtypes = [vp]
    lib.fmm_status_string.argtypes = [ctypes.c_int]
    lib.fmm_status_string.restype = ctypes.c_char_p
    lib.fmm_plan_leaves.argtypes = [vp, vp, vp, vp]
    lib.fmm_plan_cube.argtypes = [vp, dp, dp]
    lib.fmm_hilbert_index.argtypes = [ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint32, i32]
    lib.fmm_hilbert_index.restype = ctypes.c_uint64
    lib.fmm_profile_enable.argtypes = [vp, ctypes.c_int]
    lib.fmm_profile_read.argtypes = [vp, dp, ctypes.POINTER(i32)]
    lib.fmm_plan_work.argtypes = [vp, ctypes.POINTER(i64), ctypes.POINTER(i64)]
    lib.fmm_plan_tree_stats.argtypes = [vp, ctypes.POINTER(i64)]
    lib.fmm_evaluate_static.argtypes = [cfgp, i64, vp, vp, vp, vp, vp, vp, ctypes.POINTER(vp)]
    lib.fmm_replan.argtypes = [vp, vp, vp]
    lib.fmm_plan_set_schedule.argtypes = [vp, ctypes.c_int, ctypes.c_int]
    for name in EXPORTS:
        f = getattr(lib, name)
        if f.restype is ctypes.c_int or name in ("fmm_workspace_size", "fmm_plan", "fmm_evaluate",
                                                 "fmm_backward", "fmm_check", "fmm_destroy",
                                                 "fmm_plan_leaves", "fmm_plan_cube",
                                                 "fmm_profile_enable", "fmm_profile_read",
                                                 "fmm_plan_work", "fmm_plan_tree_stats",
                                                 "fmm_evaluate_static", "fmm_replan",
                                                 "fmm_plan_set_schedule"):
            f.restype = ctypes.c_int
    if path == LIB_PATH:
        _LIB = lib
    return lib


def _check(st, what):
    if st != 0:
        raise FMMError(st, what)


def make_config(p=8, depth=3, precision=FMM_PREC_FP64, lo=(0.0, 0.0, 0.0), side=1.0,
                m2l_kind=FMM_M2L_AUTO, leaf_max=0, batch_level=0):
    """leaf_max > 0 asks for the adaptive tree, depth then being its depth cap;
    batch_level > 0 makes every box of that level an independent system."""
    cfg = fmm_config()
    load().fmm_config_default(ctypes.byref(cfg))
    cfg.p, cfg.depth, cfg.precision, cfg.m2l_kind = p, depth, precision, m2l_kind
    cfg.leaf_max = leaf_max
    cfg.batch_level = batch_level
    for a in range(3):
        cfg.root_lo[a] = float(lo[a])
    cfg.root_side = float(side)
    return cfg


def fmm_workspace_size(cfg, n):
    out = ctypes.c_size_t(0)
    _check(load().fmm_workspace_size(ctypes.byref(cfg), int(n), ctypes.byref(out)),
           "fmm_workspace_size")
    return out.value


def _stream_handle(stream):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _require(t, name, dtype, numel):
    import torch
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == dtype and t.is_contiguous()
            and t.numel() == numel):
        raise ValueError(f"{name} must be a contiguous {dtype} device tensor with {numel} elements")


class Plan:
    """Handle of a plan (passed to ctypes as its pointer) with its particle
    count and device, so that the buffers given with it can be checked."""

    def __init__(self, ptr, n, device):
        self._as_parameter_ = ptr
        self.n = int(n)
        self.device = device

    @property
    def value(self):
        return self._as_parameter_.value


def fmm_plan(cfg, n, pos, workspace, stream=None):
    """pos: (n, 3) float64 device tensor; workspace: uint8 device tensor on
    the same device."""
    import torch
    _require(pos, "pos", torch.float64, 3 * n)
    if not (isinstance(workspace, torch.Tensor) and workspace.device == pos.device):
        raise ValueError("workspace must be a device tensor on the device of pos")
    plan = ctypes.c_void_p()
    _check(load().fmm_plan(ctypes.byref(cfg), int(n), _ptr(pos), _ptr(workspace),
                           workspace.numel() * workspace.element_size(), _stream_handle(stream),
                           ctypes.byref(plan)), "fmm_plan")
    return Plan(plan, n, pos.device)


def fmm_replan(plan, pos, stream=None):
    """New positions for plan (same n and configuration); keeps its operators."""
    import torch
    n = plan.n if isinstance(plan, Plan) else pos.numel() // 3
    _require_on(pos, "pos", torch.float64, 3 * n, plan)
    _check(load().fmm_replan(plan, _ptr(pos), _stream_handle(stream)), "fmm_replan")
    return plan


def fmm_plan_set_schedule(plan, key, value):
    """Work distribution of the plan's passes (FMM_SCHED_*); results are unchanged
    (M2L split: within rounding)."""
    _check(load().fmm_plan_set_schedule(plan, int(key), int(value)), "fmm_plan_set_schedule")


def _require_on(t, name, dtype, numel, plan):
    _require(t, name, dtype, numel)
    if isinstance(plan, Plan) and t.device != plan.device:
        raise ValueError(f"{name} must be on {plan.device}")


def _count(plan, t):
    """Particle count of a plan (Plan) or, for a bare pointer, of tensor t."""
    return plan.n if isinstance(plan, Plan) else t.numel()


def fmm_evaluate(plan, q, phi=None, force=None, energy=None, stream=None):
    """q: n float64 charges; phi (n), force (n, 3), energy (1): float64 outputs
    or None; all contiguous tensors on the plan's device."""
    import torch
    n = _count(plan, q)
    _require_on(q, "q", torch.float64, n, plan)
    for t, name, k in ((phi, "phi", n), (force, "force", 3 * n), (energy, "energy", 1)):
        if t is not None:
            _require_on(t, name, torch.float64, k, plan)
    _check(load().fmm_evaluate(plan, _ptr(q), _ptr(phi), _ptr(force), _ptr(energy),
                               _stream_handle(stream)), "fmm_evaluate")


def fmm_backward(plan, grad_energy, dE_dx=None, dE_dq=None, stream=None):
    """grad_energy: one float64 on the device; dE_dx (n, 3), dE_dq (n): float64
    outputs or None."""
    import torch
    _require_on(grad_energy, "grad_energy", torch.float64, 1, plan)
    n = plan.n if isinstance(plan, Plan) else (dE_dq.numel() if dE_dq is not None else
                                               (dE_dx.numel() // 3 if dE_dx is not None else 0))
    for t, name, k in ((dE_dx, "dE_dx", 3 * n), (dE_dq, "dE_dq", n)):
        if t is not None:
            _require_on(t, name, torch.float64, k, plan)
    _check(load().fmm_backward(plan, _ptr(grad_energy), _ptr(dE_dx), _ptr(dE_dq),
                               _stream_handle(stream)), "fmm_backward")


def fmm_evaluate_static(cfg, n, pos, q, phi=None, force=None, energy=None, stream=None):
    """Plan + evaluate in the library's own device scratch array (no
    allocation by the library; the outputs are the caller's).  Returns the
    library's plan for this device (valid until the next such call on it)."""
    import torch
    _require(pos, "pos", torch.float64, 3 * n)
    for t, name, k in ((q, "q", n), (phi, "phi", n), (force, "force", 3 * n), (energy, "energy", 1)):
        if t is not None:
            _require(t, name, torch.float64, k)
            if t.device != pos.device:
                raise ValueError(f"{name} must be on {pos.device}")
    plan = ctypes.c_void_p()
    _check(load().fmm_evaluate_static(ctypes.byref(cfg), int(n), _ptr(pos), _ptr(q), _ptr(phi),
                                      _ptr(force), _ptr(energy), _stream_handle(stream),
                                      ctypes.byref(plan)), "fmm_evaluate_static")
    return Plan(plan, n, pos.device)


def fmm_check(plan):
    return load().fmm_check(plan)


def fmm_destroy(plan):
    _check(load().fmm_destroy(plan), "fmm_destroy")


def fmm_status_string(status):
    return load().fmm_status_string(int(status)).decode()


def fmm_plan_leaves(plan, cells=None, leaf=None, stream=None):
    _check(load().fmm_plan_leaves(plan, _ptr(cells), _ptr(leaf), _stream_handle(stream)),
           "fmm_plan_leaves")


def fmm_plan_cube(plan):
    lo = (ctypes.c_double * 3)()
    side = ctypes.c_double()
    _check(load().fmm_plan_cube(plan, lo, ctypes.byref(side)), "fmm_plan_cube")
    return list(lo), side.value


def fmm_hilbert_index(ix, iy, iz, bits):
    return int(load().fmm_hilbert_index(ix, iy, iz, bits))


FMM_PROFILE_ALL = 0x3FF


def fmm_profile_enable(plan, on=True, phases=None):
    """Time the passes named in phases (default: every pass) while on."""
    mask = 0
    if on:
        mask = FMM_PROFILE_ALL if phases is None else sum(1 << PHASES.index(p) for p in phases)
    _check(load().fmm_profile_enable(plan, mask), "fmm_profile_enable")


def fmm_profile_read(plan):
    ms = (ctypes.c_double * len(PHASES))()
    cnt = (ctypes.c_int32 * len(PHASES))()
    _check(load().fmm_profile_read(plan, ms, cnt), "fmm_profile_read")
    return {name: (ms[i], cnt[i]) for i, name in enumerate(PHASES)}


TREE_STATS = ("boxes", "leaves", "deepest", "u", "v", "w", "x", "p2p_pairs", "m2l_pairs")


def fmm_plan_tree_stats(plan):
    """Integer statistics of an adaptive plan's tree (names in TREE_STATS)."""
    st = (ctypes.c_int64 * len(TREE_STATS))()
    _check(load().fmm_plan_tree_stats(plan, st), "fmm_plan_tree_stats")
    return dict(zip(TREE_STATS, (int(v) for v in st)))


def fmm_plan_work(plan):
    a, b = ctypes.c_int64(), ctypes.c_int64()
    _check(load().fmm_plan_work(plan, ctypes.byref(a), ctypes.byref(b)), "fmm_plan_work")
    return a.value, b.value


class FMM:
    """Owns a workspace and a plan for one position set (torch device tensors)."""

    def __init__(self, pos, p=8, depth=3, precision=FMM_PREC_FP64, lo=(0.0, 0.0, 0.0), side=1.0,
                 stream=None, workspace=None, m2l_kind=FMM_M2L_AUTO, leaf_max=0, batch_level=0):
        import torch
        self.n = pos.shape[0]
        self.cfg = make_config(p, depth, precision, lo, side, m2l_kind, leaf_max, batch_level)
        nbytes = fmm_workspace_size(self.cfg, self.n)
        if workspace is None or workspace.numel() < nbytes:
            workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=pos.device)
        off = (-workspace.data_ptr()) % 256
        self.workspace = workspace
        self._ws = workspace[off:off + nbytes]
        self.pos = pos
        self.plan = fmm_plan(self.cfg, self.n, pos, self._ws, stream)

    def evaluate(self, q, want_phi=True, want_force=True, want_energy=True, stream=None):
        import torch
        dev = q.device
        phi = torch.empty(self.n, dtype=torch.float64, device=dev) if want_phi else None
        force = torch.empty((self.n, 3), dtype=torch.float64, device=dev) if want_force else None
        energy = torch.empty(1, dtype=torch.float64, device=dev) if want_energy else None
        fmm_evaluate(self.plan, q, phi, force, energy, stream)
        return phi, force, energy

    def check(self):
        return fmm_check(self.plan)

    def close(self):
        if self.plan is not None:
            fmm_destroy(self.plan)
            self.plan = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _autograd_function():
    import torch

    class FMMEnergy(torch.autograd.Function):
        """E = 1/2 sum q_i phi_i of the FMM, differentiable in positions and
        charges through fmm_backward (dE/dq = phi, dE/dx = q grad phi, valid
        while no particle crosses a box face)."""

        @staticmethod
        def forward(ctx, pos, q, p, depth, precision, lo, side):
            # the library takes FP64 positions and charges whatever the compute
            # precision (FP32 inputs are widened here, exactly)
            f = FMM(pos.detach().to(torch.float64).contiguous(), p=p, depth=depth,
                    precision=precision, lo=lo, side=side)
            _, _, e = f.evaluate(q.detach().to(torch.float64).contiguous(), want_phi=False,
                                 want_force=False)
            st = f.check()
            if st != 0:
                f.close()
                raise FMMError(st, "fmm_evaluate (device check)")
            ctx.fmm = f
            ctx.dtypes = (pos.dtype, q.dtype)
            return e.reshape(()).to(q.dtype)

        @staticmethod
        def backward(ctx, grad_e):
            f = ctx.fmm
            g = grad_e.detach().reshape(1).to(torch.float64).contiguous()
            dx = torch.empty((f.n, 3), dtype=torch.float64, device=g.device) \
                if ctx.needs_input_grad[0] else None
            dq = torch.empty(f.n, dtype=torch.float64, device=g.device) \
                if ctx.needs_input_grad[1] else None
            if dx is not None or dq is not None:
                fmm_backward(f.plan, g, dx, dq)
                st = f.check()
                if st != 0:
                    raise FMMError(st, "fmm_backward (device check)")
            if dx is not None:
                dx = dx.to(ctx.dtypes[0])
            if dq is not None:
                dq = dq.to(ctx.dtypes[1])
            return dx, dq, None, None, None, None, None

    return FMMEnergy


_FMMENERGY = None


def fmm_energy(pos, q, p=8, depth=3, precision=FMM_PREC_FP64, lo=(0.0, 0.0, 0.0), side=1.0):
    """Differentiable FMM energy (torch.autograd) of charges q at positions pos."""
    global _FMMENERGY
    if _FMMENERGY is None:
        _FMMENERGY = _autograd_function()
    return _FMMENERGY.apply(pos, q, p, depth, precision, tuple(lo), side)
