"""Python binding of libpcfgsmc.so (argument marshalling only).

Every operation of the SMC path runs in the library's HIP kernels; this module
converts model specifications and buffers to the C interface declared in
include/pcfgsmc.h and maps status codes to exceptions. PyTorch supplies device
memory (its caching allocator, through the library's allocator callbacks) and
the HIP stream. The module refuses to run when the compiled library is absent.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libpcfgsmc.so")

OK, FINISHED = 0, 1
ERR_INVALID, ERR_OOM, ERR_DEVICE, ERR_STATE, ERR_NAN, DEGENERATE = -1, -2, -3, -4, -5, -6
STATUS_NAMES = {0: "OK", 1: "FINISHED", -1: "ERR_INVALID", -2: "ERR_OOM", -3: "ERR_DEVICE",
                -4: "ERR_STATE", -5: "ERR_NAN", -6: "DEGENERATE"}
KINDS = {"geometric": 0, "lgssm": 1, "crbd": 2, "clads": 3, "seir": 4, "crbd_ds": 5, "program": 6}
READ_BLK, READ_LW, READ_ANC, READ_FIELD0 = 0, 1, 2, 16
STOP = 255

# real fields, then int fields (see the header) per model kind
FIELDS = {
    "geometric": (0, ["flips"]),
    "lgssm": (1, ["x", "t"]),
    "crbd": (2, ["lambda", "mu", "node"]),
    "clads": (4, ["lambda", "eps", "alpha", "sigma", "node", "stack_size"]),
    "crbd_ds": (4, ["a_lambda", "th_lambda", "a_mu", "th_mu", "node"]),
    "seir": (6, ["hLambda", "hDelta", "hGamma", "mLambda", "mDelta", "rho",
                 "hS", "hE", "hI", "hR", "mS", "mE", "mI", "mR", "z", "t"]),
    # compiled programs: the stack pointer, then the stack ([particle][word], FP64)
    "program": (0, ["sp", "stack"]),
}


class SMCError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{STATUS_NAMES.get(code, code)}: {msg}")
        self.code = code


class _ProgramDesc(C.Structure):
    _fields_ = [
        ("n_blocks", C.c_uint32), ("block_start", C.POINTER(C.c_uint32)), ("code", C.POINTER(C.c_uint64)),
        ("n_code", C.c_uint32), ("consts", C.POINTER(C.c_double)), ("n_consts", C.c_uint32),
        ("data", C.POINTER(C.c_double)), ("n_data", C.c_uint32), ("array_start", C.POINTER(C.c_uint32)),
        ("n_arrays", C.c_uint32), ("stack_words", C.c_uint32),
    ]


class _Desc(C.Structure):
    _fields_ = [
        ("kind", C.c_int32), ("precision", C.c_int32), ("checkpoint", C.c_int32), ("n_nodes", C.c_int32),
        ("parent", C.POINTER(C.c_int32)), ("left", C.POINTER(C.c_int32)), ("right", C.POINTER(C.c_int32)),
        ("age", C.POINTER(C.c_double)), ("T", C.c_int32), ("y", C.POINTER(C.c_double)),
        ("params", C.c_double * 16), ("ess_threshold", C.c_double), ("program", C.POINTER(_ProgramDesc)),
    ]


def program_desc(img, keep: list) -> _ProgramDesc:
    """C description of a compiled program image (ppl.ProgramImage or a dict of
    its arrays); the arrays it points to are appended to keep."""
    get = (lambda name: img[name]) if isinstance(img, dict) else (lambda name: getattr(img, name))
    code = np.ascontiguousarray(get("code"), dtype=np.uint64)
    starts = np.ascontiguousarray(get("block_start"), dtype=np.uint32)
    consts = np.ascontiguousarray(get("consts"), dtype=np.float64)
    data = np.ascontiguousarray(get("data"), dtype=np.float64)
    astart = np.ascontiguousarray(get("array_start"), dtype=np.uint32)
    keep += [code, starts, consts, data, astart]
    d = _ProgramDesc()
    d.n_blocks = max(len(starts) - 1, 0)
    d.block_start = starts.ctypes.data_as(C.POINTER(C.c_uint32))
    d.code = code.ctypes.data_as(C.POINTER(C.c_uint64))
    d.n_code = len(code)
    d.consts = consts.ctypes.data_as(C.POINTER(C.c_double))
    d.n_consts = len(consts)
    d.data = data.ctypes.data_as(C.POINTER(C.c_double))
    d.n_data = len(data)
    d.array_start = astart.ctypes.data_as(C.POINTER(C.c_uint32))
    d.n_arrays = max(len(astart) - 1, 0)
    d.stack_words = int(get("stack_words"))
    return d


def check_program(img):
    """Validate a program image with the library's checks (no device needed):
    raises SMCError(ERR_INVALID) naming the first problem."""
    keep = []
    d = program_desc(img, keep)
    _check(lib().smc_program_check(C.byref(d)))


class _Stats(C.Structure):
    _fields_ = [("round", C.c_uint32), ("status", C.c_int32), ("block_steps", C.c_uint64),
                ("log_z", C.c_double), ("stack_depth", C.c_int32), ("resamples", C.c_uint32)]


class _KernelTimes(C.Structure):
    _fields_ = [("ms", C.c_double * 4), ("launches", C.c_uint64 * 4)]


_ALLOC = C.CFUNCTYPE(C.c_void_p, C.c_void_p, C.c_size_t)
_FREE = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p)


class _Allocator(C.Structure):
    _fields_ = [("alloc", _ALLOC), ("free", _FREE), ("ctx", C.c_void_p)]


_lib = None


def lib():
    """Load the compiled library; raise if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_2112_00364_amd.build.build()")
    L = C.CDLL(LIB_PATH)
    vp, u64, i32, u32 = C.c_void_p, C.c_uint64, C.c_int32, C.c_uint32
    sig = {
        "smc_ctx_create": [i32, vp, vp, C.POINTER(vp)],
        "smc_ctx_destroy": [vp],
        "smc_model_register": [vp, C.POINTER(_Desc), C.POINTER(vp)],
        "smc_program_check": [C.POINTER(_ProgramDesc)],
        "smc_model_destroy": [vp],
        "smc_init": [vp, u64, u64, C.POINTER(vp)],
        "smc_step": [vp], "smc_resample": [vp],
        "smc_done": [vp, C.POINTER(i32)],
        "smc_log_z": [vp, C.POINTER(C.c_double)],
        "smc_run_to_end": [vp],
        "smc_reset": [vp, u64],
        "smc_set_bucketing": [vp, i32],
        "smc_set_workgroup": [vp, i32],
        "smc_snapshot": [vp, vp, C.POINTER(C.c_size_t)],
        "smc_restore": [vp, vp, C.c_size_t],
        "smc_read": [vp, i32, vp, C.c_size_t],
        "smc_run_stats": [vp, C.POINTER(_Stats)],
        "smc_run_destroy": [vp],
        "smc_profile": [vp, i32],
        "smc_profile_read": [vp, C.POINTER(_KernelTimes)],
        "smc_resample_weights": [vp, vp, u64, u64, u32, vp, vp],
        "smc_resample_weights_noalloc": [vp, vp, u64, u64, u32, vp, vp],
        "smc_batch_create": [vp, C.POINTER(vp)],
        "smc_batch_add": [vp, vp, u64, u64, C.POINTER(i32)],
        "smc_batch_tick": [vp, i32],
        "smc_batch_set_workgroup": [vp, i32, i32],
        "smc_batch_set_owned": [vp, i32, i32],
        "smc_batch_poll": [vp, i32, vp, vp, vp, vp],
        "smc_batch_retire": [vp, i32],
        "smc_batch_destroy": [vp],
        "smc_selftest_math": [vp, i32, vp, vp, u64],
        "smc_selftest_philox": [vp, vp, vp, vp, u64],
    }
    for name, args in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = C.c_int32
    L.smc_last_error.restype = C.c_char_p
    L.smc_version.restype = C.c_char_p
    _lib = L
    return L


def _check(code, allow=(OK,)):
    if code in allow:
        return code
    raise SMCError(code, lib().smc_last_error().decode())


def _torch():
    import torch
    return torch


class Context:
    """One device and one HIP stream; device memory from torch's caching allocator."""

    def __init__(self, device: int = 0, stream=None, torch_allocator: bool = True, allocator=None):
        """allocator: optional (alloc(nbytes) -> device address or None, free(address))
        pair used instead of torch's caching allocator (None from alloc is an
        allocation failure, which the library reports as ERR_OOM)."""
        torch = _torch()
        L = lib()
        self.device = device
        torch.cuda.set_device(device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(device)
        self._alloc_ref = None
        alloc_ptr = None
        if allocator is not None:
            user_alloc, user_free = allocator

            def _a(_ctx, nbytes):
                try:
                    return user_alloc(int(nbytes))
                except Exception:
                    return None

            def _f(_ctx, p):
                user_free(p)

            self._alloc_ref = _Allocator(_ALLOC(_a), _FREE(_f), None)
            alloc_ptr = C.cast(C.pointer(self._alloc_ref), C.c_void_p)
        elif torch_allocator:
            dev, strm = device, self.stream

            def _a(_ctx, nbytes):
                try:
                    return torch.cuda.caching_allocator_alloc(int(nbytes), dev, strm)
                except Exception:
                    return None

            def _f(_ctx, p):
                torch.cuda.caching_allocator_delete(p)

            self._alloc_ref = _Allocator(_ALLOC(_a), _FREE(_f), None)
            alloc_ptr = C.cast(C.pointer(self._alloc_ref), C.c_void_p)
        h = C.c_void_p()
        _check(L.smc_ctx_create(device, C.c_void_p(self.stream.cuda_stream), alloc_ptr, C.byref(h)))
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            lib().smc_ctx_destroy(self._h)
            self._h = None

    # --- self-tests of the device primitives -------------------------------------
    def selftest_math(self, op: int, x):
        torch = _torch()
        xin = torch.as_tensor(np.ascontiguousarray(x, dtype=np.float64)).to(f"cuda:{self.device}")
        n = xin.numel() // (2 if op in (5, 6) else 3 if op in (7, 8, 10, 11, 12) else 1)
        out = torch.empty(n, dtype=torch.float64, device=xin.device)
        _check(lib().smc_selftest_math(self._h, op, C.c_void_p(xin.data_ptr()), C.c_void_p(out.data_ptr()), n))
        return out.cpu().numpy()

    def selftest_philox(self, ctr, key):
        torch = _torch()
        c = torch.as_tensor(np.ascontiguousarray(ctr, dtype=np.uint32).view(np.int32)).to(f"cuda:{self.device}")
        k = torch.as_tensor(np.ascontiguousarray(key, dtype=np.uint32).view(np.int32)).to(f"cuda:{self.device}")
        n = c.numel() // 4
        out = torch.empty(4 * n, dtype=torch.int32, device=c.device)
        _check(lib().smc_selftest_philox(self._h, C.c_void_p(c.data_ptr()), C.c_void_p(k.data_ptr()),
                                         C.c_void_p(out.data_ptr()), n))
        return out.cpu().numpy().view(np.uint32).reshape(n, 4)

    def resample_weights(self, lw, seed: int, rnd: int):
        """Resampling alone on a device (or host) log-weight vector:
        returns (status, ancestors as a uint32 numpy array, log Z increment)."""
        torch = _torch()
        t = torch.as_tensor(lw, dtype=torch.float64).to(f"cuda:{self.device}").contiguous()
        n = t.numel()
        anc = torch.zeros(n, dtype=torch.int32, device=t.device)
        inc = torch.zeros(1, dtype=torch.float64, device=t.device)
        st = lib().smc_resample_weights(self._h, C.c_void_p(t.data_ptr()), n, seed, rnd,
                                        C.c_void_p(anc.data_ptr()), C.c_void_p(inc.data_ptr()))
        _check(st, allow=(OK, DEGENERATE, ERR_NAN))
        return st, anc.cpu().numpy().view(np.uint32), float(inc.cpu()[0])

    def resample_weights_noalloc(self, lw_dev, anc_dev, inc_dev, seed: int, rnd: int) -> int:
        """smc_resample_weights_noalloc on caller-owned device tensors (float64
        log-weights, int32 ancestors of the same length, one float64 for the log
        Z increment); the library allocates nothing. Returns the status."""
        n = lw_dev.numel()
        if anc_dev.numel() < n or inc_dev.numel() < 1:
            raise ValueError("output tensors too small")
        st = lib().smc_resample_weights_noalloc(self._h, C.c_void_p(lw_dev.data_ptr()), n, seed, rnd,
                                                C.c_void_p(anc_dev.data_ptr()), C.c_void_p(inc_dev.data_ptr()))
        return _check(st, allow=(OK, DEGENERATE, ERR_NAN))


class Model:
    """A registered PCFG (Sec. 3.1) built from an input specification dict."""

    def __init__(self, ctx: Context, spec: dict):
        L = lib()
        d = _Desc()
        d.kind = KINDS[spec["kind"]]
        d.precision = int(spec.get("precision", 64))
        d.checkpoint = int(bool(spec.get("checkpoint", True)))
        self._keep = []
        tree = spec.get("tree")
        if tree is not None:
            arrs = [np.ascontiguousarray(tree[k], dtype=np.int32) for k in ("parent", "left", "right")]
            age = np.ascontiguousarray(tree["age"], dtype=np.float64)
            self._keep += arrs + [age]
            d.n_nodes = len(age)
            d.parent, d.left, d.right = (a.ctypes.data_as(C.POINTER(C.c_int32)) for a in arrs)
            d.age = age.ctypes.data_as(C.POINTER(C.c_double))
        y = spec.get("y")
        if y is not None:
            y = np.ascontiguousarray(y, dtype=np.float64)
            self._keep.append(y)
            d.T = len(y)
            d.y = y.ctypes.data_as(C.POINTER(C.c_double))
        for i, v in enumerate(spec.get("params", [])):
            d.params[i] = float(v)
        d.ess_threshold = float(spec.get("ess_threshold", 0.0))
        if spec["kind"] == "program":
            self._program = program_desc(spec["program"], self._keep)
            d.program = C.pointer(self._program)
        h = C.c_void_p()
        _check(L.smc_model_register(ctx._h, C.byref(d), C.byref(h)))
        self._h = h
        self.ctx = ctx
        self.spec = spec
        self.kind = spec["kind"]
        self.precision = d.precision

    def close(self):
        if getattr(self, "_h", None):
            if self.ctx._h is not None:  # after the context is gone its memory is gone too
                lib().smc_model_destroy(self._h)
            self._h = None


class Run:
    """One SMC run: init (Alg. 1 step 1), then step / resample."""

    def __init__(self, model: Model, n: int, seed: int):
        h = C.c_void_p()
        _check(lib().smc_init(model._h, int(n), int(seed), C.byref(h)))
        self._h = h
        self.model = model
        self.n = int(n)

    def step(self):
        return _check(lib().smc_step(self._h), allow=(OK, FINISHED, DEGENERATE))

    def resample(self):
        return _check(lib().smc_resample(self._h), allow=(OK, FINISHED, DEGENERATE))

    def done(self):
        d = C.c_int32()
        st = _check(lib().smc_done(self._h, C.byref(d)), allow=(OK, FINISHED, DEGENERATE, ERR_NAN))
        return bool(d.value), st

    def log_z(self):
        v = C.c_double()
        _check(lib().smc_log_z(self._h, C.byref(v)), allow=(OK, FINISHED, DEGENERATE, ERR_NAN))
        return v.value

    def run_to_end(self):
        return _check(lib().smc_run_to_end(self._h), allow=(FINISHED, DEGENERATE))

    def reset(self, seed: int):
        _check(lib().smc_reset(self._h, int(seed)))

    def snapshot(self) -> bytes:
        """The run's complete state as bytes (checkpoint)."""
        size = C.c_size_t(0)
        _check(lib().smc_snapshot(self._h, None, C.byref(size)))
        buf = C.create_string_buffer(size.value)
        _check(lib().smc_snapshot(self._h, C.cast(buf, C.c_void_p), C.byref(size)))
        return buf.raw[:size.value]

    def restore(self, snap: bytes):
        """Load a snapshot of a run of the same model and size (resume)."""
        buf = C.create_string_buffer(snap, len(snap))
        _check(lib().smc_restore(self._h, C.cast(buf, C.c_void_p), len(snap)))

    def set_workgroup(self, lanes: int):
        """Lanes per propagation work-group, 128 or 256 (results unchanged)."""
        _check(lib().smc_set_workgroup(self._h, int(lanes)))

    def set_bucketing(self, enable: bool = True):
        """Sort particle slots by resume block before each propagation (results unchanged)."""
        _check(lib().smc_set_bucketing(self._h, 1 if enable else 0))

    def stats(self):
        s = _Stats()
        _check(lib().smc_run_stats(self._h, C.byref(s)))
        return {"round": s.round, "status": s.status, "block_steps": s.block_steps, "log_z": s.log_z,
                "stack_depth": s.stack_depth, "resamples": s.resamples}

    def profile(self, enable: bool = True):
        _check(lib().smc_profile(self._h, 1 if enable else 0))

    def kernel_times(self):
        """{kernel: (total ms, launches)} for propagate, bucketing (three launches per
        entry), reduce (+ fold_sums) and scan_anc."""
        t = _KernelTimes()
        _check(lib().smc_profile_read(self._h, C.byref(t)))
        names = ("propagate", "bucket", "reduce", "scan_anc")
        return {names[i]: (t.ms[i], int(t.launches[i])) for i in range(4)}

    def _read(self, what, dtype, count=1):
        out = np.zeros(self.n * count, dtype=dtype)
        _check(lib().smc_read(self._h, what, out.ctypes.data_as(C.c_void_p), out.nbytes))
        return out

    def blk(self):
        return self._read(READ_BLK, np.uint8)

    def lw(self):
        return self._read(READ_LW, np.float64)

    def anc(self):
        return self._read(READ_ANC, np.uint32)

    def field(self, k, dtype, count=1):
        out = self._read(READ_FIELD0 + k, dtype, count)
        return out if count == 1 else out.reshape(self.n, count)

    def close(self):
        if getattr(self, "_h", None):
            if self.model.ctx._h is not None:  # a run outliving its context is only forgotten
                lib().smc_run_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Many independent runs advanced together."""

    def __init__(self, ctx: Context):
        h = C.c_void_p()
        _check(lib().smc_batch_create(ctx._h, C.byref(h)))
        self._h = h
        self.ctx = ctx
        self.n_slots = 0

    def add(self, model: Model, n: int, seed: int) -> int:
        slot = C.c_int32()
        _check(lib().smc_batch_add(self._h, model._h, int(n), int(seed), C.byref(slot)))
        self.n_slots = max(self.n_slots, slot.value + 1)
        return slot.value

    def tick(self, rounds: int = 1):
        _check(lib().smc_batch_tick(self._h, int(rounds)))

    def set_workgroup(self, slot: int, lanes: int):
        """Lanes per propagation work-group of one run of the batch (128 or 256;
        results unchanged)."""
        _check(lib().smc_batch_set_workgroup(self._h, int(slot), int(lanes)))

    def set_owned(self, slot: int, owned: bool = True):
        """One work-group advances this run through every round of a tick
        (built-in models of at most 4096 particles; results unchanged)."""
        _check(lib().smc_batch_set_owned(self._h, int(slot), 1 if owned else 0))

    def poll(self):
        k = self.n_slots
        done = np.zeros(k, dtype=np.int32)
        lz = np.zeros(k, dtype=np.float64)
        st = np.zeros(k, dtype=np.int32)
        steps = np.zeros(k, dtype=np.uint64)
        _check(lib().smc_batch_poll(self._h, k, done.ctypes.data_as(C.c_void_p), lz.ctypes.data_as(C.c_void_p),
                                    st.ctypes.data_as(C.c_void_p), steps.ctypes.data_as(C.c_void_p)))
        return done.astype(bool), lz, st, steps

    def retire(self, slot: int):
        _check(lib().smc_batch_retire(self._h, int(slot)))

    def close(self):
        if getattr(self, "_h", None):
            if self.ctx._h is not None:
                lib().smc_batch_destroy(self._h)
            self._h = None
