"""ctypes wrapper around the CPU oracle (smc_oracle.c) -- test infrastructure.

Only the test suite, the smoke check and the CPU-baseline leg of the benchmark
may import this module. It shares no code with the GPU library: it takes plain
arrays and a model specification (a dict of inputs) and drives Algorithm 1 of
Lunden et al. (Sec. 3.2) one step at a time in single-threaded C.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "smc_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")
CFLAGS = ["-O2", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared", "-std=c11",
          "-Wall", "-Wextra"]

KINDS = {"geometric": 0, "lgssm": 1, "crbd": 2, "clads": 3, "seir": 4, "crbd_ds": 5}
STOP = 255
OK, FINISHED, ERR_INVALID, ERR_NAN, DEGENERATE = 0, 1, -1, -5, -6
READ_BLK, READ_LW, READ_ANC, READ_FIELD0 = 0, 1, 2, 16


def build() -> str:
    """Compile the oracle with gcc (always recompiles)."""
    tmp = f"{LIB}.{os.getpid()}.tmp"  # per process: concurrent builds do not collide
    subprocess.run(["gcc", *CFLAGS, "-o", tmp, SRC, "-lm"], check=True)
    os.replace(tmp, LIB)
    return LIB


class _Model(C.Structure):
    _fields_ = [
        ("kind", C.c_int32), ("precision", C.c_int32), ("checkpoint", C.c_int32),
        ("n_nodes", C.c_int32),
        ("parent", C.POINTER(C.c_int32)), ("left", C.POINTER(C.c_int32)),
        ("right", C.POINTER(C.c_int32)), ("age", C.POINTER(C.c_double)),
        ("T", C.c_int32), ("y", C.POINTER(C.c_double)),
        ("p", C.c_double * 16),
        ("ess_threshold", C.c_double),
    ]


_lib = None


def lib():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        build()
    L = C.CDLL(LIB)
    u32p, u64p, f64p = C.POINTER(C.c_uint32), C.POINTER(C.c_uint64), C.POINTER(C.c_double)
    L.or_philox4x32_10.argtypes = [u32p, u32p, u32p]
    L.or_exp.argtypes = [C.c_double]; L.or_exp.restype = C.c_double
    L.or_log.argtypes = [C.c_double]; L.or_log.restype = C.c_double
    L.or_cos2pi.argtypes = [C.c_double]; L.or_cos2pi.restype = C.c_double
    L.or_word.argtypes = [C.c_uint64, C.c_uint32, C.c_uint32, C.c_uint32, C.c_uint32]
    L.or_word.restype = C.c_uint32
    L.or_uniform_from_word.argtypes = [C.c_uint32]; L.or_uniform_from_word.restype = C.c_double
    L.or_poisson_words.argtypes = [C.c_double, u32p, C.c_int32, C.POINTER(C.c_int32)]
    L.or_poisson_words.restype = C.c_int64
    L.or_log_factorial.argtypes = [C.c_int64]; L.or_log_factorial.restype = C.c_double
    L.or_log_binomial_pmf.argtypes = [C.c_int64, C.c_int64, C.c_double]; L.or_log_binomial_pmf.restype = C.c_double
    L.or_sample.argtypes = [C.c_int32, C.c_double, C.c_double, C.c_uint64, C.c_int64, f64p]
    L.or_draw.argtypes = [C.c_int32, C.c_double, C.c_double, C.c_uint64, C.c_uint32, C.c_uint32, u32p,
                          C.POINTER(C.c_int32)]
    L.or_draw.restype = C.c_double
    L.or_ancestors.argtypes = [u64p, C.c_uint64, C.c_uint32, u32p]
    L.or_systematic.argtypes = [f64p, C.c_uint64, C.c_uint64, C.c_uint32, u32p, f64p, u64p]
    L.or_systematic.restype = C.c_int32
    L.or_create.argtypes = [C.POINTER(_Model), C.c_uint64, C.c_uint64]; L.or_create.restype = C.c_void_p
    L.or_destroy.argtypes = [C.c_void_p]
    for name in ("or_step", "or_resample", "or_run_to_end", "or_status", "or_max_stack"):
        getattr(L, name).argtypes = [C.c_void_p]
        getattr(L, name).restype = C.c_int32
    L.or_log_z.argtypes = [C.c_void_p]; L.or_log_z.restype = C.c_double
    L.or_round.argtypes = [C.c_void_p]; L.or_round.restype = C.c_uint32
    L.or_block_steps.argtypes = [C.c_void_p]; L.or_block_steps.restype = C.c_uint64
    L.or_resamples.argtypes = [C.c_void_p]; L.or_resamples.restype = C.c_uint32
    L.or_ess_resamples.argtypes = [f64p, C.c_uint64, C.c_double]; L.or_ess_resamples.restype = C.c_int32
    L.or_read.argtypes = [C.c_void_p, C.c_int32, C.c_void_p]; L.or_read.restype = C.c_int32
    L.or_propagate_particle.argtypes = [C.POINTER(_Model), C.c_uint64, C.c_uint32, C.c_uint32,
                                        C.POINTER(C.c_uint8), f64p, f64p, C.POINTER(C.c_int32), f64p]
    L.or_propagate_particle.restype = C.c_int32
    _lib = L
    return L


def _ptr(a, ctype):
    return a.ctypes.data_as(C.POINTER(ctype))


# --- primitives -----------------------------------------------------------

def philox(ctr, key):
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    lib().or_philox4x32_10(_ptr(c, C.c_uint32), _ptr(k, C.c_uint32), _ptr(out, C.c_uint32))
    return out


def word(seed, k, particle, rnd, tag):
    return int(lib().or_word(seed, k, particle, rnd, tag))


def exp(x):
    return lib().or_exp(float(x))


def log(x):
    return lib().or_log(float(x))


def cos2pi(u):
    return lib().or_cos2pi(float(u))


def uniform_from_word(w):
    return lib().or_uniform_from_word(int(w))


def poisson_words(m, words):
    w = np.ascontiguousarray(words, dtype=np.uint32)
    used = C.c_int32(0)
    k = lib().or_poisson_words(float(m), _ptr(w, C.c_uint32), len(w), C.byref(used))
    return int(k), int(used.value)


def ancestors(Q, U):
    Q = np.ascontiguousarray(Q, dtype=np.uint64)
    anc = np.zeros(len(Q), dtype=np.uint32)
    lib().or_ancestors(_ptr(Q, C.c_uint64), len(Q), int(U), _ptr(anc, C.c_uint32))
    return anc


def systematic(lw, seed, rnd):
    """Resample one log-weight vector: (status, ancestors, log Z increment, total grid units)."""
    lw = np.ascontiguousarray(lw, dtype=np.float64)
    anc = np.zeros(len(lw), dtype=np.uint32)
    inc = C.c_double(0.0)
    qtot = C.c_uint64(0)
    st = lib().or_systematic(_ptr(lw, C.c_double), len(lw), seed, rnd, _ptr(anc, C.c_uint32),
                             C.byref(inc), C.byref(qtot))
    return int(st), anc, inc.value, int(qtot.value)


def log_factorial(k):
    return lib().or_log_factorial(int(k))


def log_binomial_pmf(y, z, p):
    return lib().or_log_binomial_pmf(int(y), int(z), float(p))


def sample(kind, a, b, seed, count):
    """count draws from one stream: kind "binomial" (n=a, p=b), "gamma" (shape a), "beta" (a, b),
    "negbin" (Poisson count with rate ~ Gamma(a, scale b)), "lomax" (Exponential lifetime with
    rate ~ Gamma(a, scale b))."""
    out = np.zeros(int(count), dtype=np.float64)
    code = {"binomial": 0, "gamma": 1, "beta": 2, "negbin": 3, "lomax": 4}[kind]
    lib().or_sample(code, float(a), float(b), int(seed), int(count), _ptr(out, C.c_double))
    return out


def draw(dist, a, b, seed, particle, rnd, k):
    """One program draw (or_draw): returns (value, next word index, fault flag)."""
    kk = C.c_uint32(int(k))
    fault = C.c_int32(0)
    v = lib().or_draw(int(dist), float(a), float(b), int(seed), int(particle), int(rnd), C.byref(kk),
                      C.byref(fault))
    return v, int(kk.value), bool(fault.value)


def ess_resamples(lw, threshold):
    """The ESS rule on one log-weight vector: 1 resample, 0 carry, -1 invalid threshold."""
    lw = np.ascontiguousarray(lw, dtype=np.float64)
    return int(lib().or_ess_resamples(_ptr(lw, C.c_double), len(lw), float(threshold)))


# --- runs -----------------------------------------------------------------

def _model_struct(spec, keep):
    m = _Model()
    m.kind = KINDS[spec["kind"]]
    m.precision = int(spec.get("precision", 64))
    m.checkpoint = int(bool(spec.get("checkpoint", True)))
    tree = spec.get("tree")
    if tree is not None:
        arrs = {k: np.ascontiguousarray(tree[k], dtype=np.int32) for k in ("parent", "left", "right")}
        age = np.ascontiguousarray(tree["age"], dtype=np.float64)
        keep += list(arrs.values()) + [age]
        m.n_nodes = len(age)
        m.parent = _ptr(arrs["parent"], C.c_int32)
        m.left = _ptr(arrs["left"], C.c_int32)
        m.right = _ptr(arrs["right"], C.c_int32)
        m.age = _ptr(age, C.c_double)
    y = spec.get("y")
    if y is not None:
        y = np.ascontiguousarray(y, dtype=np.float64)
        keep.append(y)
        m.T = len(y)
        m.y = _ptr(y, C.c_double)
    for i, v in enumerate(spec.get("params", [])):
        m.p[i] = float(v)
    m.ess_threshold = float(spec.get("ess_threshold", 0.0))
    return m


N_REAL = {"geometric": 0, "lgssm": 1, "crbd": 2, "clads": 4, "seir": 6, "crbd_ds": 4}
N_INT = {"geometric": 1, "lgssm": 1, "crbd": 1, "clads": 2, "seir": 10, "crbd_ds": 1}


def propagate_particle(spec, seed, slot, rnd, blk, reals, ints, stack=None, stack_depth=0):
    """Run one particle's blocks for round `rnd` in slot `slot` from the given state.
    Returns (blk, lw, reals, ints, stack)."""
    keep = []
    m = _model_struct(spec, keep)
    b = C.c_uint8(int(blk))
    lw = C.c_double(0.0)
    r = np.zeros(max(1, N_REAL[spec["kind"]]), dtype=np.float64)
    r[:len(reals)] = reals
    i = np.zeros(max(1, N_INT[spec["kind"]]), dtype=np.int32)
    i[:len(ints)] = ints
    st = None
    if stack is not None:
        st = np.zeros(stack_depth, dtype=np.float64)
        st[:len(stack)] = stack
    code = lib().or_propagate_particle(C.byref(m), int(seed), int(slot), int(rnd), C.byref(b), C.byref(lw),
                                       _ptr(r, C.c_double), _ptr(i, C.c_int32),
                                       _ptr(st, C.c_double) if st is not None else None)
    if code != OK:
        raise ValueError("oracle rejected the particle")
    return int(b.value), lw.value, r, i, st


class Run:
    """One SMC run of Algorithm 1 on the CPU oracle."""

    def __init__(self, spec: dict, n: int, seed: int):
        L = lib()
        m = _Model()
        m.kind = KINDS[spec["kind"]]
        m.precision = int(spec.get("precision", 64))
        m.checkpoint = int(bool(spec.get("checkpoint", True)))
        self._keep = []
        tree = spec.get("tree")
        if tree is not None:
            arrs = {k: np.ascontiguousarray(tree[k], dtype=np.int32) for k in ("parent", "left", "right")}
            age = np.ascontiguousarray(tree["age"], dtype=np.float64)
            self._keep += list(arrs.values()) + [age]
            m.n_nodes = len(age)
            m.parent = _ptr(arrs["parent"], C.c_int32)
            m.left = _ptr(arrs["left"], C.c_int32)
            m.right = _ptr(arrs["right"], C.c_int32)
            m.age = _ptr(age, C.c_double)
        y = spec.get("y")
        if y is not None:
            y = np.ascontiguousarray(y, dtype=np.float64)
            self._keep.append(y)
            m.T = len(y)
            m.y = _ptr(y, C.c_double)
        params = list(spec.get("params", []))
        for i, v in enumerate(params):
            m.p[i] = float(v)
        m.ess_threshold = float(spec.get("ess_threshold", 0.0))
        self._m = m
        self.n = int(n)
        self.spec = spec
        self._h = L.or_create(C.byref(m), self.n, int(seed))
        if not self._h:
            raise ValueError("oracle rejected the model or particle count")

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            lib().or_destroy(h)
            self._h = None

    def step(self):
        return int(lib().or_step(self._h))

    def resample(self):
        return int(lib().or_resample(self._h))

    def run_to_end(self):
        return int(lib().or_run_to_end(self._h))

    @property
    def log_z(self):
        return lib().or_log_z(self._h)

    @property
    def status(self):
        return int(lib().or_status(self._h))

    @property
    def round(self):
        return int(lib().or_round(self._h))

    @property
    def block_steps(self):
        return int(lib().or_block_steps(self._h))

    @property
    def resamples(self):
        return int(lib().or_resamples(self._h))

    @property
    def max_stack(self):
        return int(lib().or_max_stack(self._h))

    def blk(self):
        out = np.zeros(self.n, dtype=np.uint8)
        lib().or_read(self._h, READ_BLK, out.ctypes.data_as(C.c_void_p))
        return out

    def lw(self):
        out = np.zeros(self.n, dtype=np.float64)
        lib().or_read(self._h, READ_LW, out.ctypes.data_as(C.c_void_p))
        return out

    def anc(self):
        out = np.zeros(self.n, dtype=np.uint32)
        lib().or_read(self._h, READ_ANC, out.ctypes.data_as(C.c_void_p))
        return out

    def field(self, k, dtype, count=1):
        out = np.zeros(self.n * count, dtype=dtype)
        st = lib().or_read(self._h, READ_FIELD0 + k, out.ctypes.data_as(C.c_void_p))
        if st != OK:
            raise IndexError(k)
        return out if count == 1 else out.reshape(self.n, count)
