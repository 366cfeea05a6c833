"""Python binding of libemx (box-constrained Euclidean median by EM-ADMM on
MI355X / gfx950).

Argument marshalling only: every step of the solve runs in the HIP kernels
of ``libemx.so`` (see ``include/emx.h`` for the C ABI).  PyTorch supplies
device memory and the current stream.  Importing this module does not load
the library; the first call does, and raises ``RuntimeError`` if the library
was not built (there is no CPU fallback).
"""

from __future__ import annotations

import ctypes as C
import os
import threading

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("EMX_LIBRARY") or os.path.join(HERE, "libemx.so")

EM_OK, EM_ERR_INVALID_ARG, EM_ERR_UNSUPPORTED, EM_ERR_OUT_OF_MEMORY, EM_ERR_HIP = 0, -1, -2, -3, -4
CONVERGED, MAXITER, EMPTY, BAD_INPUT = 1, 2, 4, 8
RESTART_SHIFT = 8   # accelerated ADMM: flags >> RESTART_SHIFT = restarts
INIT_GIVEN, INIT_MAXW, INIT_WMEAN = 0, 1, 2
SOLVER_ADMM, SOLVER_IRLS, SOLVER_ADMM_ADAPTIVE, SOLVER_ADMM_FAST, SOLVER_ADMM_WEIGHTED = 0, 1, 2, 3, 4
SET_BOX, SET_BALL = 0, 1
NLEM_INIT_NOISY, NLEM_INIT_NLM = 0, 1
MAX_D, MAX_N, MAX_PATCH_RADIUS, MAX_WINDOW_RADIUS = 64, 512, 3, 10
NOALLOC_MAX_PIXELS = 1 << 22   # nlem_denoise_noalloc: largest H * W

# the 16-byte per-instance / per-pixel result record (em_stats_t)
STATS_FIELDS = ("iters", "flags", "r_pri", "r_dual")


class EmxError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{msg} (status {status})")
        self.status = status


class NlemImage(C.Structure):
    _fields_ = [("img", C.c_void_p), ("out", C.c_void_p), ("stats", C.c_void_p),
                ("H", C.c_int32), ("W", C.c_int32), ("patch_radius", C.c_int32),
                ("window_radius", C.c_int32), ("h_param", C.c_float), ("img_is_f16", C.c_int32)]


class NlemOptions(C.Structure):
    _fields_ = [("solver", C.c_int32), ("init", C.c_int32), ("lo", C.c_float), ("hi", C.c_float),
                ("rho", C.c_float), ("eps", C.c_float), ("max_iter", C.c_int32), ("tol", C.c_float)]


PLAN_BUILTIN, PLAN_TUNED, PLAN_CACHE, PLAN_SET = 0, 1, 2, 3
PLAN_SOURCES = ("builtin", "tuned", "cache", "set")


class NlemPlan(C.Structure):
    """nlem_plan_t: schedule of the NLEM solve kernel for one shape."""
    _fields_ = [("waves", C.c_int32), ("chunk", C.c_int32), ("order", C.c_int32),
                ("arm_factor", C.c_float), ("check_every", C.c_int32), ("source", C.c_int32)]

    def as_dict(self):
        return dict(waves=self.waves, chunk=self.chunk, order=self.order,
                    arm_factor=float(self.arm_factor), check_every=self.check_every,
                    source=PLAN_SOURCES[self.source])


class BatchPlan(C.Structure):
    """em_batch_plan_t: sliced classes routed to the generic kernels, arm factor."""
    _fields_ = [("generic_classes", C.c_uint64), ("arm_factor", C.c_float), ("check_every", C.c_int32),
                ("host_counts", C.c_int32), ("source", C.c_int32)]

    def as_dict(self):
        return dict(generic_classes=int(self.generic_classes), arm_factor=float(self.arm_factor),
                    check_every=self.check_every, host_counts=self.host_counts,
                    source=PLAN_SOURCES[self.source])


class EmOptions(C.Structure):
    _fields_ = [("solver", C.c_int32), ("init", C.c_int32), ("lo", C.c_float), ("hi", C.c_float),
                ("box_lo", C.c_void_p), ("box_hi", C.c_void_p), ("rho", C.c_float),
                ("eps", C.c_float), ("max_iter", C.c_int32), ("tol", C.c_float),
                ("adapt_every", C.c_int32), ("adapt_ratio", C.c_float), ("adapt_factor", C.c_float),
                ("fast_eta", C.c_float), ("set", C.c_int32), ("ball_center", C.c_void_p),
                ("ball_radius", C.c_void_p), ("radius", C.c_float), ("points_f16", C.c_int32)]


_lib = None
_lib_lock = threading.Lock()


def load_library():
    """Load libemx.so (built by ``build()``); raises if it is missing."""
    global _lib
    with _lib_lock:
        if _lib is not None:
            return _lib
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} not found: build the HIP library first "
                               "(python -c 'import __graft_entry__ as g; g.build()')")
        # torch first: it brings its own HIP runtime (same soname as the system
        # one), and libemx.so must bind to that runtime, not load a second one
        # that torch would then pick up in place of its own.
        import torch  # noqa: F401
        lib = C.CDLL(LIB_PATH)
        vp, i32, i64, f32 = C.c_void_p, C.c_int32, C.c_int64, C.c_float
        lib.em_create.argtypes = [C.POINTER(vp), C.c_int]
        lib.em_create.restype = C.c_int
        lib.em_destroy.argtypes = [vp]
        lib.em_destroy.restype = C.c_int
        lib.em_solve_batch.argtypes = [vp, vp, i64, vp, vp, vp, f32, f32, f32, i32, f32, i32, vp, vp]
        lib.em_solve_batch.restype = C.c_int
        lib.em_solve_batch_ex.argtypes = [vp, vp, i64, vp, vp, vp, C.POINTER(EmOptions), vp, vp]
        lib.em_solve_batch_ex.restype = C.c_int
        lib.em_solve_plain_ex.argtypes = [vp, vp, i64, vp, vp, vp, vp, C.POINTER(EmOptions), vp, vp]
        lib.em_solve_plain_ex.restype = C.c_int
        lib.em_solve_plain.argtypes = [vp, vp, i64, vp, vp, vp, vp, f32, f32, f32, i32, f32, i32, vp, vp]
        lib.em_solve_plain.restype = C.c_int
        lib.nlem_denoise.argtypes = [vp, vp, vp, i32, i32, i32, i32, i32, f32, f32, f32, f32, i32, f32,
                                     vp, vp]
        lib.nlem_denoise.restype = C.c_int
        lib.nlem_denoise_noalloc.argtypes = lib.nlem_denoise.argtypes
        lib.nlem_denoise_noalloc.restype = C.c_int
        lib.nlem_denoise_multi.argtypes = [vp, vp, i32, C.POINTER(NlemImage), f32, f32, f32, i32, f32]
        lib.nlem_denoise_multi.restype = C.c_int
        lib.nlem_denoise_ex.argtypes = [vp, vp, i32, C.POINTER(NlemImage), C.POINTER(NlemOptions)]
        lib.nlem_denoise_ex.restype = C.c_int
        lib.nlm_denoise.argtypes = [vp, vp, vp, i32, i32, i32, i32, i32, f32, vp]
        lib.nlm_denoise.restype = C.c_int
        lib.nlem_autotune.argtypes = [vp, vp, C.POINTER(NlemImage), C.POINTER(NlemOptions), i32,
                                      C.POINTER(i32)]
        lib.nlem_autotune.restype = C.c_int
        lib.nlem_plan.argtypes = [vp, i32, i32, i32, C.POINTER(i32)]
        lib.nlem_plan.restype = C.c_int
        lib.nlem_plan_get.argtypes = [vp, i32, i32, i32, i32, C.POINTER(NlemPlan)]
        lib.nlem_plan_get.restype = C.c_int
        lib.nlem_plan_set.argtypes = [vp, i32, i32, i32, i32, C.POINTER(NlemPlan)]
        lib.nlem_plan_set.restype = C.c_int
        lib.em_batch_autotune.argtypes = [vp, vp, i64, vp, vp, vp, C.POINTER(EmOptions), vp, vp, i32,
                                          C.POINTER(BatchPlan)]
        lib.em_batch_autotune.restype = C.c_int
        lib.em_batch_plan_get.argtypes = [vp, i32, i32, C.POINTER(BatchPlan)]
        lib.em_batch_plan_get.restype = C.c_int
        lib.em_batch_plan_set.argtypes = [vp, i32, i32, C.POINTER(BatchPlan)]
        lib.em_batch_plan_set.restype = C.c_int
        lib.em_kernel_timing.argtypes = [vp, i32]
        lib.em_kernel_timing.restype = C.c_int
        lib.em_kernel_timing_read.argtypes = [vp, C.POINTER(C.c_double), C.POINTER(i64)]
        lib.em_kernel_timing_read.restype = C.c_int
        lib.em_sync.argtypes = [vp, vp]
        lib.em_sync.restype = C.c_int
        lib.em_status_string.argtypes = [C.c_int]
        lib.em_status_string.restype = C.c_char_p
        lib.em_last_error.argtypes = [vp]
        lib.em_last_error.restype = C.c_char_p
        _lib = lib
        return lib


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _stream(stream):
    if stream is not None:
        return C.c_void_p(stream)
    import torch
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


class Handle:
    """An em_handle_t bound to one device (see em_create)."""

    def __init__(self, device: int = 0):
        self.lib = load_library()
        self.device = device
        h = C.c_void_p()
        st = self.lib.em_create(C.byref(h), int(device))
        if st != EM_OK:
            raise EmxError(st, f"em_create(device={device}) failed")
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            self.lib.em_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, st: int, what: str):
        if st != EM_OK:
            msg = self.lib.em_last_error(self.h).decode()
            raise EmxError(st, f"{what}: {self.lib.em_status_string(st).decode()} {msg}")

    # -- calls ----------------------------------------------------------------

    def em_solve_batch(self, a, w, inst, z, stats=None, *, lo, hi, rho, max_iter, tol,
                       init=INIT_MAXW, stream=None):
        """a, w: float32 device tensors; inst: device tensor of em_instance_t
        (B x 32 bytes, e.g. an int64 tensor of shape [B, 4]); z: float32 device
        tensor (in/out); stats: None or an int32/float32 device tensor of
        B x 4 words."""
        B = int(inst.numel() * inst.element_size() // 32)
        st = self.lib.em_solve_batch(self.h, _stream(stream), B, _ptr(a), _ptr(w), _ptr(inst),
                                     float(lo), float(hi), float(rho), int(max_iter), float(tol),
                                     int(init), _ptr(z), _ptr(stats))
        self._check(st, "em_solve_batch")

    def em_solve_batch_ex(self, a, w, inst, z, stats=None, *, solver=SOLVER_ADMM, init=INIT_MAXW,
                          lo=-float("inf"), hi=float("inf"), box_lo=None, box_hi=None, rho=1.0,
                          eps=1e-6, max_iter=1000, tol=1e-4, adapt_every=1, adapt_ratio=10.0,
                          adapt_factor=2.0, ball_center=None, ball_radius=None, radius=None,
                          eta=0.999, stream=None):
        """em_solve_batch with a solver choice (ADMM, IRLS, adaptive-penalty ADMM,
        accelerated ADMM with restart parameter eta, weighted-penalty ADMM)
        and a general set: per-coordinate bounds box_lo / box_hi (float32 device
        tensors laid out like z), or the Euclidean ball when `radius` (scalar)
        or `ball_radius` (one per instance) is given, centred at ball_center
        (laid out like z; origin when None).  A float16 tensor `a` is passed
        as FP16 point storage."""
        B = int(inst.numel() * inst.element_size() // 32)
        opt = _options(solver, init, lo, hi, box_lo, box_hi, rho, eps, max_iter, tol, adapt_every,
                       adapt_ratio, adapt_factor, eta, ball_center, ball_radius, radius)
        import torch
        opt.points_f16 = 1 if a.dtype == torch.float16 else 0
        st = self.lib.em_solve_batch_ex(self.h, _stream(stream), B, _ptr(a), _ptr(w), _ptr(inst),
                                        C.byref(opt), _ptr(z), _ptr(stats))
        self._check(st, "em_solve_batch_ex")

    def em_solve_plain_ex(self, a, w, inst, inst_host, z, stats=None, *, solver=SOLVER_ADMM,
                          init=INIT_MAXW, lo=-float("inf"), hi=float("inf"), box_lo=None, box_hi=None,
                          rho=1.0, max_iter=1000, tol=1e-4, eta=0.999, stream=None):
        """em_solve_plain with options: solver SOLVER_ADMM or SOLVER_ADMM_FAST
        (accelerated ADMM with restart parameter eta), optional per-coordinate
        bounds."""
        B = int(inst.numel() * inst.element_size() // 32)
        hp = inst_host.ctypes.data if hasattr(inst_host, "ctypes") else inst_host.data_ptr()
        opt = _options(solver, init, lo, hi, box_lo, box_hi, rho, 1e-6, max_iter, tol, 1, 10.0, 2.0, eta)
        import torch
        opt.points_f16 = 1 if a.dtype == torch.float16 else 0
        st = self.lib.em_solve_plain_ex(self.h, _stream(stream), B, _ptr(a), _ptr(w), _ptr(inst),
                                        C.c_void_p(hp), C.byref(opt), _ptr(z), _ptr(stats))
        self._check(st, "em_solve_plain_ex")

    def em_solve_plain(self, a, w, inst, inst_host, z, stats=None, *, lo, hi, rho, max_iter, tol,
                       init=INIT_MAXW, stream=None):
        """As em_solve_batch, one launch per instance; inst_host is the same
        descriptor array in host memory (numpy array or CPU tensor)."""
        B = int(inst.numel() * inst.element_size() // 32)
        hp = inst_host.ctypes.data if hasattr(inst_host, "ctypes") else inst_host.data_ptr()
        st = self.lib.em_solve_plain(self.h, _stream(stream), B, _ptr(a), _ptr(w), _ptr(inst),
                                     C.c_void_p(hp), float(lo), float(hi), float(rho),
                                     int(max_iter), float(tol), int(init), _ptr(z), _ptr(stats))
        self._check(st, "em_solve_plain")

    def nlem_denoise(self, img, out, stats=None, *, patch_radius, window_radius, h, lo=0.0,
                     hi=255.0, rho=1e-3, max_iter=200, tol=1e-4, stream=None):
        """img: H x W float32 or float16 device tensor; out: H x W float32."""
        import torch
        H, W = int(img.shape[0]), int(img.shape[1])
        is16 = 1 if img.dtype == torch.float16 else 0
        st = self.lib.nlem_denoise(self.h, _stream(stream), _ptr(img), is16, H, W,
                                   int(patch_radius), int(window_radius), float(h), float(lo),
                                   float(hi), float(rho), int(max_iter), float(tol), _ptr(out),
                                   _ptr(stats))
        self._check(st, "nlem_denoise")

    def nlem_denoise_noalloc(self, img, out, stats=None, *, patch_radius, window_radius, h, lo=0.0,
                             hi=255.0, rho=1e-3, max_iter=200, tol=1e-4, stream=None):
        """nlem_denoise with the library's static scratch instead of handle
        workspace (no device allocation; H * W <= NOALLOC_MAX_PIXELS)."""
        import torch
        H, W = int(img.shape[0]), int(img.shape[1])
        is16 = 1 if img.dtype == torch.float16 else 0
        st = self.lib.nlem_denoise_noalloc(self.h, _stream(stream), _ptr(img), is16, H, W,
                                           int(patch_radius), int(window_radius), float(h),
                                           float(lo), float(hi), float(rho), int(max_iter),
                                           float(tol), _ptr(out), _ptr(stats))
        self._check(st, "nlem_denoise_noalloc")

    def nlem_denoise_multi(self, items, *, lo=0.0, hi=255.0, rho=1e-3, max_iter=200, tol=1e-4,
                           stream=None):
        """items: list of dicts with img, out, stats (optional), patch_radius,
        window_radius, h."""
        arr = _image_array(items)
        self._keep = (arr, items)  # descriptors must outlive graph (re)creation
        st = self.lib.nlem_denoise_multi(self.h, _stream(stream), len(items), arr, float(lo),
                                         float(hi), float(rho), int(max_iter), float(tol))
        self._check(st, "nlem_denoise_multi")

    def nlem_denoise_ex(self, items, *, solver=SOLVER_ADMM, init=NLEM_INIT_NOISY, lo=0.0, hi=255.0,
                        rho=1e-3, eps=1e-6, max_iter=200, tol=1e-4, stream=None):
        """items: list of dicts with img, out, stats (optional), patch_radius,
        window_radius, h (as nlem_denoise_multi)."""
        arr = _image_array(items)
        opt = NlemOptions(int(solver), int(init), float(lo), float(hi), float(rho), float(eps),
                          int(max_iter), float(tol))
        st = self.lib.nlem_denoise_ex(self.h, _stream(stream), len(items), arr, C.byref(opt))
        self._check(st, "nlem_denoise_ex")

    def nlem_autotune(self, item, *, solver=SOLVER_ADMM, init=NLEM_INIT_NOISY, lo=0.0, hi=255.0,
                      rho=1e-3, eps=1e-6, max_iter=200, tol=1e-4, repeats=2, stream=None):
        """Search the schedule of this image's shape (coordinate waves, queue
        chunk, queue order, residual arm factor) on the image (a dict as for
        nlem_denoise_ex) and keep the fastest plan; returns its coordinate-wave
        count (the whole plan: nlem_plan_get)."""
        arr = _image_array([item])
        opt = NlemOptions(int(solver), int(init), float(lo), float(hi), float(rho), float(eps),
                          int(max_iter), float(tol))
        chosen = C.c_int32(0)
        st = self.lib.nlem_autotune(self.h, _stream(stream), arr, C.byref(opt), int(repeats),
                                    C.byref(chosen))
        self._check(st, "nlem_autotune")
        return chosen.value

    def nlem_plan(self, patch_radius, window_radius, solver=SOLVER_ADMM):
        """Coordinate-wave count used for this shape and solver."""
        waves = C.c_int32(0)
        self._check(self.lib.nlem_plan(self.h, int(patch_radius), int(window_radius), int(solver),
                                       C.byref(waves)), "nlem_plan")
        return waves.value

    def nlem_plan_get(self, patch_radius, window_radius, solver=SOLVER_ADMM, f16=False):
        """The whole plan (dict: waves, chunk, order, arm_factor, source)."""
        p = NlemPlan()
        self._check(self.lib.nlem_plan_get(self.h, int(patch_radius), int(window_radius), int(solver),
                                           1 if f16 else 0, C.byref(p)), "nlem_plan_get")
        return p.as_dict()

    def nlem_plan_set(self, patch_radius, window_radius, plan=None, solver=SOLVER_ADMM, f16=False):
        """Set the plan (dict with waves, chunk, order, arm_factor, check_every)
        or, with plan=None, return to the built-in one."""
        p = None if plan is None else NlemPlan(int(plan["waves"]), int(plan.get("chunk", 0)),
                                               int(plan.get("order", -1)),
                                               float(plan.get("arm_factor", 1.0)),
                                               int(plan.get("check_every", 1)), 0)
        self._check(self.lib.nlem_plan_set(self.h, int(patch_radius), int(window_radius), int(solver),
                                           1 if f16 else 0, None if p is None else C.byref(p)),
                    "nlem_plan_set")

    def em_batch_autotune(self, a, w, inst, z, stats=None, *, lo, hi, rho, max_iter, tol,
                          init=INIT_MAXW, box_lo=None, box_hi=None, repeats=2, stream=None):
        """Tune the batched fixed-penalty EM-ADMM over a box on this batch;
        returns the chosen plan (dict)."""
        import torch
        B = int(inst.numel() * inst.element_size() // 32)
        opt = _options(SOLVER_ADMM, init, lo, hi, box_lo, box_hi, rho, 1e-6, max_iter, tol, 1, 10.0,
                       2.0, 0.999)
        opt.points_f16 = 1 if a.dtype == torch.float16 else 0
        p = BatchPlan()
        st = self.lib.em_batch_autotune(self.h, _stream(stream), B, _ptr(a), _ptr(w), _ptr(inst),
                                        C.byref(opt), _ptr(z), _ptr(stats), int(repeats), C.byref(p))
        self._check(st, "em_batch_autotune")
        return p.as_dict()

    def em_batch_plan_get(self, f16=False, solver=SOLVER_ADMM):
        p = BatchPlan()
        self._check(self.lib.em_batch_plan_get(self.h, int(solver), 1 if f16 else 0, C.byref(p)),
                    "em_batch_plan_get")
        return p.as_dict()

    def em_batch_plan_set(self, plan=None, f16=False, solver=SOLVER_ADMM):
        """Set the batch plan (dict with generic_classes, arm_factor,
        check_every, host_counts) or, with plan=None, return to the built-in
        one."""
        p = None if plan is None else BatchPlan(int(plan.get("generic_classes", 0)),
                                                float(plan.get("arm_factor", 1.0)),
                                                int(plan.get("check_every", 1)),
                                                int(plan.get("host_counts", 0)), 0)
        self._check(self.lib.em_batch_plan_set(self.h, int(solver), 1 if f16 else 0,
                                               None if p is None else C.byref(p)), "em_batch_plan_set")

    def nlm_denoise(self, img, out, *, patch_radius, window_radius, h, stream=None):
        """Non-Local Means: img H x W float32/float16, out H x W float32."""
        import torch
        H, W = int(img.shape[0]), int(img.shape[1])
        is16 = 1 if img.dtype == torch.float16 else 0
        st = self.lib.nlm_denoise(self.h, _stream(stream), _ptr(img), is16, H, W, int(patch_radius),
                                  int(window_radius), float(h), _ptr(out))
        self._check(st, "nlm_denoise")

    def kernel_timing(self, enable=True):
        """Bracket every NLEM solve launch with HIP events (em_kernel_timing)."""
        self._check(self.lib.em_kernel_timing(self.h, 1 if enable else 0), "em_kernel_timing")

    def kernel_timing_read(self):
        """(summed milliseconds, launches) of the timed NLEM solve launches since
        the last read; waits for them."""
        ms = C.c_double(0.0)
        n = C.c_int64(0)
        self._check(self.lib.em_kernel_timing_read(self.h, C.byref(ms), C.byref(n)), "em_kernel_timing_read")
        return ms.value, n.value

    def sync(self, stream=None):
        self._check(self.lib.em_sync(self.h, _stream(stream)), "em_sync")


def _options(solver, init, lo, hi, box_lo, box_hi, rho, eps, max_iter, tol, adapt_every, adapt_ratio,
             adapt_factor, eta, ball_center=None, ball_radius=None, radius=None):
    ball = radius is not None or ball_radius is not None
    return EmOptions(int(solver), int(init), float(lo), float(hi),
                     None if box_lo is None else box_lo.data_ptr(),
                     None if box_hi is None else box_hi.data_ptr(), float(rho), float(eps),
                     int(max_iter), float(tol), int(adapt_every), float(adapt_ratio),
                     float(adapt_factor), float(eta), SET_BALL if ball else SET_BOX,
                     None if ball_center is None else ball_center.data_ptr(),
                     None if ball_radius is None else ball_radius.data_ptr(),
                     float(0.0 if radius is None else radius), 0)


def _image_array(items):
    import torch
    arr = (NlemImage * len(items))()
    for k, it in enumerate(items):
        img = it["img"]
        arr[k] = NlemImage(img.data_ptr(), it["out"].data_ptr(),
                           it["stats"].data_ptr() if it.get("stats") is not None else None,
                           int(img.shape[0]), int(img.shape[1]), int(it["patch_radius"]),
                           int(it["window_radius"]), float(it["h"]),
                           1 if img.dtype == torch.float16 else 0)
    return arr


_handles = {}


def handle(device: int = 0) -> Handle:
    """A process-wide handle per device."""
    h = _handles.get(device)
    if h is None:
        h = _handles[device] = Handle(device)
    return h


def stats_view(stats):
    """Split a B x 4 int32 stats tensor into (iters, flags, r_pri, r_dual)."""
    import torch
    s = stats.view(torch.int32).reshape(-1, 4)
    return s[:, 0], s[:, 1], s[:, 2].view(torch.float32), s[:, 3].view(torch.float32)


def instances_tensor(inst_np, device="cuda"):
    """Upload a numpy em_instance_t array (synth.pointsets.INSTANCE_DTYPE) as a
    [B, 4] int64 device tensor with the same bytes."""
    import numpy as np
    import torch
    raw = np.ascontiguousarray(inst_np).view(np.int64).reshape(-1, 4)
    return torch.from_numpy(raw.copy()).to(device)
