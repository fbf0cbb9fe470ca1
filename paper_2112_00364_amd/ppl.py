"""Front end for CorePPL-style programs: source text -> PCFG bytecode (Sec. 4).

The library runs universal programs registered as PCFGs whose blocks are
bytecode (SMC_MODEL_PROGRAM in include/pcfgsmc.h). This module is the host
tool that produces them, following the compilation scheme of Sec. 4:

1. parse the source (s-expressions, below);
2. static analysis (Sec. 4.3): a function is *decomposed* when it contains a
   resample, calls a decomposed function, or is recursive. The bytecode has no
   native call stack, so recursive resample-free functions also keep their
   frames on the program-state stack (the paper leaves those to the C
   compiler);
3. every other function is inlined at its call sites;
4. the body of each decomposed function is classified into the statement
   kinds of eq. (3) and split into basic blocks by Algorithm 2 (`decompose`);
5. stack frames as in Sec. 4.1: each decomposed function has a frame of
   fixed size holding its return block, the location of its return value,
   its parameters and every local that more than one block uses (a local used
   by a single block lives in a register of that block, as Sec. 4.1 allows;
   call results stay in the frame, since the callee writes them there); the
   caller allocates the whole frame and
   writes the first three parts before jumping to the callee; addresses on the
   stack are relative to the stack base, since resampling moves particles
   (Sec. 4.3);
6. code generation to the bytecode of the library's program interpreter.

Source language. A program is `(program ITEM ...)` with items

    (data NAME v ...)              constant array of numbers
    (def NAME (PARAM ...) STMT ...) function; `main` (no parameters) is the entry

and statements, in the A-normal form the decomposition assumes (Sec. 4.1:
calls, draws and checkpoints bind names; expressions are pure):

    (let X E)                      X := E
    (sample X DIST E ...)          X ~ DIST(E ...)
    (observe DIST E ... V)         log-weight += log p_DIST(V | E ...)
    (weight E)                     log-weight += E
    (resample)                     SMC checkpoint (Sec. 4.1)
    (if E (STMT ...) (STMT ...))   branch on E != 0
    (call X F E ...)               X := F(E ...)
    (return E)                     in tail position only: the last statement of the
                                   body, or of a branch of an if in tail position

Expressions: numbers, names, `(OP E ...)` with OP in + - * / neg < <= > >=
== != not log exp sqrt floor, `(at NAME E)` (element E of a data array) and
`(len NAME)`. Comparisons give 1 or 0. Distributions and their arguments:
uniform (a, b), normal (mean, sd), exponential (rate), gamma (shape >= 1,
scale), beta (a >= 1, b >= 1), bernoulli (p), poisson (mean), binomial (n, p);
gamma and beta cannot be observed. A path without a return returns 0.

Tail calls: a function that calls itself and returns the result at once
(`(call X F ...)` then `(return X)`, in tail position) reuses its own frame:
the arguments overwrite the parameters and control jumps back to the entry
block, so a recursion over observations keeps a constant stack. (Alg. 2
expresses such a call as a `call` whose next block is `return`.)
"""
from __future__ import annotations

import itertools
from dataclasses import dataclass, field

import numpy as np

# ---------------------------------------------------------------------------
# Bytecode (the interpreter in csrc/program.hpp executes it; the header
# include/pcfgsmc.h documents every instruction). One 64-bit word per
# instruction: op | x << 8 | y << 16 | z << 24 | imm << 32.
# ---------------------------------------------------------------------------
OPS = {
    "FRAME": 1, "CONST": 2, "IMM": 3, "MOV": 4, "LDF": 5, "STF": 6,
    "ADD": 7, "SUB": 8, "MUL": 9, "DIV": 10, "LT": 11, "LE": 12, "EQ": 13, "NE": 14,
    "NEG": 15, "NOT": 16, "LOG": 17, "EXP": 18, "SQRT": 19, "FLOOR": 20,
    "DATA": 21, "LEN": 22, "SAMPLE": 23, "OBSERVE": 24, "WEIGHT": 25,
    "JZ": 26, "JMP": 27, "CALLFRAME": 28, "STN": 29, "ADDR": 30, "PUSH": 31,
    "STRET": 32, "GOTO": 33, "CKPT": 34, "JRET": 35, "FAULT": 36,
}
TERMINATORS = {"GOTO", "CKPT", "JRET", "FAULT"}
N_REGS = 16
REG_LOCALS = 8  # block-local variables held in registers per block (r15 downwards)
STOP = 255
MAX_BLOCKS = 254

# distribution ids and argument counts
DISTS = {"uniform": (0, 2), "normal": (1, 2), "exponential": (2, 1), "gamma": (3, 2), "beta": (4, 2),
         "bernoulli": (5, 1), "poisson": (6, 1), "binomial": (7, 2)}
OBSERVABLE = {"uniform", "normal", "exponential", "bernoulli", "poisson", "binomial"}

BINARY = {"+": "ADD", "-": "SUB", "*": "MUL", "/": "DIV", "<": "LT", "<=": "LE", "==": "EQ", "!=": "NE"}
SWAPPED = {">": "LT", ">=": "LE"}  # a > b is b < a
UNARY = {"neg": "NEG", "not": "NOT", "log": "LOG", "exp": "EXP", "sqrt": "SQRT", "floor": "FLOOR"}


class CompileError(ValueError):
    pass


# ---------------------------------------------------------------------------
# Parsing
# ---------------------------------------------------------------------------
def _tokens(text):
    out = []
    for line in text.splitlines():
        line = line.split(";", 1)[0]
        out += line.replace("(", " ( ").replace(")", " ) ").split()
    return out


def _read(tokens, i):
    if i >= len(tokens):
        raise CompileError("unexpected end of program text")
    t = tokens[i]
    if t == ")":
        raise CompileError("unbalanced ')'")
    if t != "(":
        return t, i + 1
    items, i = [], i + 1
    while i < len(tokens) and tokens[i] != ")":
        v, i = _read(tokens, i)
        items.append(v)
    if i >= len(tokens):
        raise CompileError("missing ')'")
    return items, i + 1


def _number(t):
    try:
        return float(t)
    except (TypeError, ValueError):
        return None


def _expr(x):
    if isinstance(x, str):
        v = _number(x)
        return ("num", v) if v is not None else ("var", x)
    if not x:
        raise CompileError("empty expression")
    head, args = x[0], x[1:]
    if head == "at" and len(args) == 2 and isinstance(args[0], str):
        return ("at", args[0], _expr(args[1]))
    if head == "len" and len(args) == 1 and isinstance(args[0], str):
        return ("len", args[0])
    if head in BINARY or head in SWAPPED:
        if len(args) != 2:
            raise CompileError(f"'{head}' takes two operands")
        return ("op", head, [_expr(a) for a in args])
    if head in UNARY:
        if len(args) != 1:
            raise CompileError(f"'{head}' takes one operand")
        return ("op", head, [_expr(args[0])])
    raise CompileError(f"unknown expression {x!r}")


def _name(x, what):
    if not isinstance(x, str) or _number(x) is not None:
        raise CompileError(f"{what} must be a name, got {x!r}")
    return x


def _stmt(x):
    if not isinstance(x, list) or not x:
        raise CompileError(f"statement expected, got {x!r}")
    h, a = x[0], x[1:]
    if h == "let" and len(a) == 2:
        return ("let", _name(a[0], "let target"), _expr(a[1]))
    if h == "sample" and len(a) >= 2:
        d = DISTS.get(a[1])
        if d is None or len(a) - 2 != d[1]:
            raise CompileError(f"bad sample statement {x!r}")
        return ("sample", _name(a[0], "sample target"), a[1], [_expr(e) for e in a[2:]])
    if h == "observe" and len(a) >= 2:
        d = DISTS.get(a[0])
        if d is None or a[0] not in OBSERVABLE or len(a) - 2 != d[1]:
            raise CompileError(f"bad observe statement {x!r}")
        return ("observe", a[0], [_expr(e) for e in a[1:-1]], _expr(a[-1]))
    if h == "weight" and len(a) == 1:
        return ("weight", _expr(a[0]))
    if h == "resample" and not a:
        return ("resample",)
    if h == "if" and len(a) == 3 and isinstance(a[1], list) and isinstance(a[2], list):
        return ("if", _expr(a[0]), [_stmt(s) for s in a[1]], [_stmt(s) for s in a[2]])
    if h == "call" and len(a) >= 2:
        return ("call", _name(a[0], "call target"), _name(a[1], "function"), [_expr(e) for e in a[2:]])
    if h == "return" and len(a) == 1:
        return ("return", _expr(a[0]))
    raise CompileError(f"unknown statement {x!r}")


@dataclass
class Function:
    name: str
    params: list
    body: list


@dataclass
class Source:
    functions: dict
    data: dict  # name -> list of floats, in declaration order


def parse(text: str) -> Source:
    toks = _tokens(text)
    tree, i = _read(toks, 0)
    if i != len(toks):
        raise CompileError("text after the program")
    if not isinstance(tree, list) or not tree or tree[0] != "program":
        raise CompileError("a program starts with (program ...)")
    funcs, data = {}, {}
    for item in tree[1:]:
        if not isinstance(item, list) or not item:
            raise CompileError(f"bad program item {item!r}")
        if item[0] == "data" and len(item) >= 2:
            vals = [_number(v) for v in item[2:]]
            if any(v is None for v in vals):
                raise CompileError(f"data {item[1]} holds a non-number")
            data[_name(item[1], "data name")] = vals
        elif item[0] == "def" and len(item) >= 3 and isinstance(item[2], list):
            name = _name(item[1], "function name")
            if name in funcs:
                raise CompileError(f"function {name} defined twice")
            params = [_name(p, "parameter") for p in item[2]]
            body = [_stmt(s) for s in item[3:]]
            if not _returns_in_tail_only(body, True):
                raise CompileError(f"{name}: return only in tail position")
            funcs[name] = Function(name, params, body)
        else:
            raise CompileError(f"bad program item {item!r}")
    if "main" not in funcs or funcs["main"].params:
        raise CompileError("the program needs a main function without parameters")
    return Source(funcs, data)


# ---------------------------------------------------------------------------
# Static analysis (Sec. 4.3) and inlining
# ---------------------------------------------------------------------------
def _walk(stmts):
    for s in stmts:
        yield s
        if s[0] == "if":
            yield from _walk(s[2])
            yield from _walk(s[3])


def _returns_in_tail_only(stmts, tail):
    """Is every return the last statement of a list in tail position?"""
    for k, s in enumerate(stmts):
        last = tail and k == len(stmts) - 1
        if s[0] == "return" and not last:
            return False
        if s[0] == "if" and not all(_returns_in_tail_only(b, last) for b in (s[2], s[3])):
            return False
    return True


def _end_paths(stmts, on_return, on_fallthrough):
    """Rewrites how every path of a tail-position list ends: a final return
    through on_return(expression), a final if branch by branch, anything else
    by appending on_fallthrough()."""
    if stmts and stmts[-1][0] == "return":
        return stmts[:-1] + on_return(stmts[-1][1])
    if stmts and stmts[-1][0] == "if":
        s = stmts[-1]
        return stmts[:-1] + [("if", s[1], _end_paths(s[2], on_return, on_fallthrough),
                              _end_paths(s[3], on_return, on_fallthrough))]
    return stmts + on_fallthrough()


# A self tail call's arguments are held in registers while the parameters are
# rewritten; beyond this many they go through temporary frame slots instead.
MAX_TAIL_ARGS = N_REGS - REG_LOCALS


def _tail_calls(f, params, stmts):
    """`(call X f ...)` followed by `(return X)` at the end of a tail-position
    list -> `(tailcall f ...)` (self-calls only)."""
    if len(stmts) >= 2 and stmts[-1][0] == "return" and stmts[-2][0] == "call":
        c = stmts[-2]
        if c[2] == f and stmts[-1][1] == ("var", c[1]):
            return stmts[:-2] + [("tailcall", f, c[3])]
    if stmts and stmts[-1][0] == "if":
        s = stmts[-1]
        return stmts[:-1] + [("if", s[1], _tail_calls(f, params, s[2]), _tail_calls(f, params, s[3]))]
    return stmts


def decomposed_functions(src: Source) -> set:
    calls = {f: {s[2] for s in _walk(fn.body) if s[0] == "call"} for f, fn in src.functions.items()}
    for f, cs in calls.items():
        for g in cs:
            if g not in src.functions:
                raise CompileError(f"{f} calls unknown function {g}")
        for s in _walk(src.functions[f].body):
            if s[0] == "call" and len(s[3]) != len(src.functions[s[2]].params):
                raise CompileError(f"{f} calls {s[2]} with the wrong number of arguments")
    # recursive: f reaches itself through calls
    def reaches(a, b):
        seen, todo = set(), [a]
        while todo:
            x = todo.pop()
            for y in calls[x]:
                if y == b:
                    return True
                if y not in seen:
                    seen.add(y)
                    todo.append(y)
        return False

    dec = {f for f, fn in src.functions.items()
           if f == "main" or any(s[0] == "resample" for s in _walk(fn.body)) or reaches(f, f)}
    changed = True
    while changed:
        changed = False
        for f in src.functions:
            if f not in dec and calls[f] & dec:
                dec.add(f)
                changed = True
    return dec


def _rename_expr(e, ren):
    k = e[0]
    if k == "num" or k == "len":
        return e
    if k == "var":
        return ("var", ren.get(e[1], e[1]))
    if k == "at":
        return ("at", e[1], _rename_expr(e[2], ren))
    return ("op", e[1], [_rename_expr(a, ren) for a in e[2]])


def _rename_stmt(s, ren):
    k = s[0]
    r = lambda e: _rename_expr(e, ren)  # noqa: E731
    if k == "let":
        return ("let", ren[s[1]], r(s[2]))
    if k == "sample":
        return ("sample", ren[s[1]], s[2], [r(e) for e in s[3]])
    if k == "observe":
        return ("observe", s[1], [r(e) for e in s[2]], r(s[3]))
    if k == "weight":
        return ("weight", r(s[1]))
    if k == "if":
        return ("if", r(s[1]), [_rename_stmt(t, ren) for t in s[2]], [_rename_stmt(t, ren) for t in s[3]])
    if k == "call":
        return ("call", ren[s[1]], s[2], [r(e) for e in s[3]])
    if k == "return":
        return ("return", r(s[1]))
    return s


def _assigned(stmts):
    out = []
    for s in _walk(stmts):
        if s[0] in ("let", "sample", "call") and s[1] not in out:
            out.append(s[1])
    return out


def inline(src: Source, dec: set) -> dict:
    """Bodies of the decomposed functions with every call to a non-decomposed
    function replaced by the callee's body (renamed, parameters bound first)."""
    site = itertools.count()

    def expand(stmts):
        out = []
        for s in stmts:
            if s[0] == "call" and s[2] not in dec:
                g = src.functions[s[2]]
                tag = f"{g.name}#{next(site)}."
                ren = {v: tag + v for v in g.params + _assigned(g.body)}
                out += [("let", ren[p], a) for p, a in zip(g.params, s[3])]
                body = [_rename_stmt(t, ren) for t in g.body]
                target = s[1]
                body = _end_paths(body, lambda e, t=target: [("let", t, e)],
                                  lambda t=target: [("let", t, ("num", 0.0))])
                out += expand(body)
            elif s[0] == "if":
                out.append(("if", s[1], expand(s[2]), expand(s[3])))
            else:
                out.append(s)
        return out

    result = {}
    for f in src.functions:
        if f in dec:
            body = expand(src.functions[f].body)
            result[f] = _end_paths(body, lambda e: [("return", e)], lambda: [("return", ("num", 0.0))])
    return result


def _expr_vars(e, out):
    k = e[0]
    if k == "var":
        out.add(e[1])
    elif k == "at":
        _expr_vars(e[2], out)
    elif k == "op":
        for a in e[2]:
            _expr_vars(a, out)
    return out


def _stmt_names(s, out):
    """Names one statement defines or reads (an if: its condition only)."""
    k = s[0]
    if k in ("let", "sample", "call"):
        out.add(s[1])
    if k == "let":
        _expr_vars(s[2], out)
    elif k in ("sample", "call"):
        for e in s[3]:
            _expr_vars(e, out)
    elif k == "observe":
        for e in s[2] + [s[3]]:
            _expr_vars(e, out)
    elif k in ("weight", "return", "if"):
        _expr_vars(s[1], out)
    elif k == "tailcall":
        for e in s[2]:
            _expr_vars(e, out)
    return out


def _block_names(items, out):
    for it in items:
        if it[0] == "other":
            _stmt_names(it[1], out)
        elif it[0] == "call":
            _stmt_names(it[2], out)
        elif it[0] == "if":
            _stmt_names(it[1], out)
            _block_names(it[2], out)
            _block_names(it[3], out)
    return out


def _check_defined(name, body, params):
    """Every name is assigned on every path before it is read."""
    def go(stmts, defined):
        for s in stmts:
            used = set()
            k = s[0]
            if k in ("let", "weight", "return"):
                _expr_vars(s[2] if k == "let" else s[1], used)
            elif k in ("sample", "call"):
                for e in s[3]:
                    _expr_vars(e, used)
            elif k == "observe":
                for e in s[2] + [s[3]]:
                    _expr_vars(e, used)
            elif k == "if":
                _expr_vars(s[1], used)
            elif k == "tailcall":
                for e in s[2]:
                    _expr_vars(e, used)
            missing = used - defined
            if missing:
                raise CompileError(f"{name}: {sorted(missing)[0]} may be read before it is assigned")
            if k in ("let", "sample", "call"):
                defined = defined | {s[1]}
            elif k == "if":
                defined = go(s[2], defined) & go(s[3], defined)
        return defined

    go(body, set(params))


# ---------------------------------------------------------------------------
# Algorithm 2: function decomposition into basic blocks.
# Statements are classified as checkpoint, call, if or other (eq. (3)); the
# result (eq. (4)) tags checkpoints and calls with the block that follows
# them, adds jumps, and maps block indices to statement lists. `nxt` is the
# accumulator's third component: None (nothing to do at the end of the
# block), RETURN (the return block of the current call) or a block index.
# ---------------------------------------------------------------------------
RETURN = "return"


class Decomposer:
    def __init__(self, kind, counter):
        self.kind = kind        # statement -> "checkpoint" | "call" | "if" | "other"
        self.counter = counter  # shared source of fresh block indices (newIndex)
        self.branches = lambda s: (s[2], s[3])

    def fresh(self):
        return next(self.counter)

    def first_split(self, nxt):  # initNext
        return self.fresh() if nxt is None else nxt

    def decompose(self, stmts):
        block, blocks, _ = self.rec([], {}, RETURN, list(stmts))
        entry = self.fresh()
        blocks = dict(blocks)
        blocks[entry] = block
        return entry, blocks

    def rec(self, block, blocks, nxt, stmts):
        if not stmts:
            if nxt is None:
                return block, blocks, nxt
            return block + [("jump", nxt)], blocks, nxt
        s, rest = stmts[0], stmts[1:]
        k = self.kind(s)
        if k in ("checkpoint", "call"):
            if not rest:
                nxt = self.first_split(nxt)
                return block + [(k, nxt, s)], blocks, nxt
            index = self.fresh()
            following, blocks, nxt = self.rec([], blocks, self.first_split(nxt), rest)
            return block + [(k, index, s)], {**blocks, index: following}, nxt
        if k == "other":
            return self.rec(block + [("other", s)], blocks, nxt, rest)
        thn_src, els_src = self.branches(s)
        if not rest:  # if in tail position: both branches end the block
            thn, blocks, t_next = self.rec([], blocks, nxt, thn_src)
            els, blocks, e_next = self.rec([], blocks, t_next, els_src)
            if nxt != e_next and t_next is None:
                thn = thn + [("jump", e_next)]
            return block + [("if", s, thn, els)], blocks, e_next
        thn, blocks, t_next = self.rec([], blocks, None, thn_src)
        els, blocks, e_next = self.rec([], blocks, t_next, els_src)
        if e_next is None:  # no split in either branch: the if stays inside the block
            return self.rec(block + [("if", s, thn, els)], blocks, nxt, rest)
        if t_next is None:
            thn = thn + [("jump", e_next)]
        following, blocks, nxt = self.rec([], blocks, self.first_split(nxt), rest)
        return block + [("if", s, thn, els)], {**blocks, e_next: following}, nxt


def decompose_abstract(stmts, first_index=1):
    """Algorithm 2 on the abstract statements of eq. (3): 'other', 'checkpoint',
    'call' or ('if', [...], [...]). Returns (entry index, {index: block})."""
    def kind(s):
        return "if" if isinstance(s, tuple) else s

    d = Decomposer(kind, itertools.count(first_index))
    d.branches = lambda s: (s[1], s[2])
    return d.decompose(stmts)


# ---------------------------------------------------------------------------
# Code generation
# ---------------------------------------------------------------------------
@dataclass
class ProgramImage:
    """Everything smc_model_register needs for SMC_MODEL_PROGRAM."""
    code: np.ndarray          # uint64 instructions
    block_start: np.ndarray   # uint32 [n_blocks + 1]
    consts: np.ndarray        # float64
    data: np.ndarray          # float64, all arrays concatenated
    array_start: np.ndarray   # uint32 [n_arrays + 1]
    stack_words: int          # stack capacity per particle (8-byte words)
    block_names: list = field(default_factory=list)  # for listings: "function:index"
    frames: dict = field(default_factory=dict)       # function -> frame words
    entry: dict = field(default_factory=dict)        # function -> entry block

    @property
    def n_blocks(self):
        return len(self.block_start) - 1


def _enc(op, x=0, y=0, z=0, imm=0):
    return OPS[op] | (x << 8) | (y << 16) | (z << 24) | ((imm & 0xFFFFFFFF) << 32)


class _Gen:
    def __init__(self, src: Source, frames, slots, entries, block_of):
        self.src = src
        self.frames = frames
        self.slots = slots
        self.entries = entries
        self.block_of = block_of  # Alg. 2 index -> final block number
        self.consts = []
        self.const_ix = {}
        self.arrays = list(src.data)
        self.regs = {}          # block-local variable -> register, for the block being generated
        self.limit = N_REGS     # expression registers are those below the first local's

    def const(self, v):
        key = np.float64(v).tobytes()
        if key not in self.const_ix:
            self.const_ix[key] = len(self.consts)
            self.consts.append(float(v))
        return self.const_ix[key]

    def array(self, name):
        if name not in self.src.data:
            raise CompileError(f"unknown data array {name}")
        return self.arrays.index(name)

    # expressions: value into register r; registers above r are scratch
    def expr(self, e, r, f, out):
        if r >= self.limit:
            raise CompileError(f"{f}: expression too deep for {self.limit} registers")
        k = e[0]
        if k == "num":
            out.append(["CONST", r, 0, 0, self.const(e[1])])
        elif k == "var":
            if e[1] in self.regs:
                out.append(["MOV", r, self.regs[e[1]], 0, 0])
            elif e[1] in self.slots[f]:
                out.append(["LDF", r, 0, 0, self.slots[f][e[1]]])
            else:
                raise CompileError(f"{f}: unknown name {e[1]}")
        elif k == "at":
            self.expr(e[2], r, f, out)
            out.append(["DATA", r, r, 0, self.array(e[1])])
        elif k == "len":
            out.append(["LEN", r, 0, 0, self.array(e[1])])
        else:
            op, args = e[1], e[2]
            if op in UNARY:
                self.expr(args[0], r, f, out)
                out.append([UNARY[op], r, r, 0, 0])
            else:
                a, b = (args[1], args[0]) if op in SWAPPED else (args[0], args[1])
                self.expr(a, r, f, out)
                self.expr(b, r + 1, f, out)
                out.append([SWAPPED.get(op) or BINARY[op], r, r, r + 1, 0])

    def store(self, name, f, out):
        """r0 -> variable (its register, or its frame slot)."""
        if name in self.regs:
            out.append(["MOV", self.regs[name], 0, 0, 0])
        else:
            out.append(["STF", 0, 0, 0, self.slots[f][name]])

    def stmt(self, s, f, out):
        k = s[0]
        if k == "let":
            self.expr(s[2], 0, f, out)
            self.store(s[1], f, out)
        elif k == "sample":
            for i, e in enumerate(s[3]):
                self.expr(e, i, f, out)
            out.append(["SAMPLE", 0, 0, 1, DISTS[s[2]][0]])
            self.store(s[1], f, out)
        elif k == "observe":
            for i, e in enumerate(s[2]):
                self.expr(e, i, f, out)
            self.expr(s[3], 2, f, out)
            out.append(["OBSERVE", 2, 0, 1, DISTS[s[1]][0]])
        elif k == "weight":
            self.expr(s[1], 0, f, out)
            out.append(["WEIGHT", 0, 0, 0, 0])
        elif k == "return":
            self.expr(s[1], 0, f, out)
            out.append(["STRET", 0, 0, 0, 0])
        else:
            raise CompileError(f"internal: statement {k} reached code generation")

    def tstmts(self, items, f, out):
        for it in items:
            k = it[0]
            if k == "other":
                self.stmt(it[1], f, out)
            elif k == "checkpoint":
                if it[1] == RETURN:
                    raise CompileError("internal: checkpoint returns")
                out.append(["CKPT", 0, 0, 0, self.block_of[it[1]]])
            elif k == "call":
                s = it[2]
                if s[0] == "tailcall":
                    # self tail call: arguments to registers, then over the
                    # parameters, and back to the entry block with the same frame
                    if it[1] != RETURN:
                        raise CompileError("internal: tail call not in tail position")
                    params = self.src.functions[f].params
                    if len(s[2]) <= min(MAX_TAIL_ARGS, self.limit):
                        for i, e in enumerate(s[2]):
                            self.expr(e, i, f, out)
                        for i, p in enumerate(params):
                            out.append(["STF", i, 0, 0, self.slots[f][p]])
                    else:  # through the frame's tail temporaries
                        for i, e in enumerate(s[2]):
                            self.expr(e, 0, f, out)
                            out.append(["STF", 0, 0, 0, self.slots[f][f"$tail{i}"]])
                        for i, p in enumerate(params):
                            out.append(["LDF", 0, 0, 0, self.slots[f][f"$tail{i}"]])
                            out.append(["STF", 0, 0, 0, self.slots[f][p]])
                    out.append(["GOTO", 0, 0, 0, self.entries[f]])
                    continue
                if it[1] == RETURN:
                    raise CompileError("internal: tail call")
                g, fr = s[2], self.frames[s[2]]
                out.append(["CALLFRAME", 0, 0, 0, fr])
                out.append(["IMM", 0, 0, 0, self.block_of[it[1]]])
                out.append(["STN", 0, 0, 0, 0])
                out.append(["ADDR", 0, 0, 0, self.slots[f][s[1]]])
                out.append(["STN", 0, 0, 0, 1])
                for i, e in enumerate(s[3]):
                    self.expr(e, 0, f, out)
                    out.append(["STN", 0, 0, 0, 2 + i])
                out.append(["PUSH", 0, 0, 0, fr])
                out.append(["GOTO", 0, 0, 0, self.entries[g]])
            elif k == "jump":
                if it[1] == RETURN:
                    out.append(["JRET", 0, 0, 0, self.frames[f]])
                else:
                    out.append(["GOTO", 0, 0, 0, self.block_of[it[1]]])
            elif k == "if":
                self.expr(it[1][1], 0, f, out)
                jz = ["JZ", 0, 0, 0, None]
                out.append(jz)
                self.tstmts(it[2], f, out)
                jmp = ["JMP", 0, 0, 0, None]
                out.append(jmp)
                jz[4] = len(out)
                self.tstmts(it[3], f, out)
                jmp[4] = len(out)
            else:
                raise CompileError(f"internal: {k}")


def _kind(dec):
    def kind(s):
        if s[0] == "resample":
            return "checkpoint"
        if s[0] in ("call", "tailcall"):
            return "call"  # inlining left only calls of decomposed functions
        if s[0] == "if":
            return "if"
        return "other"
    return kind


def compile_program(text: str, stack_words: int = 256) -> ProgramImage:
    """Source text -> bytecode image (blocks numbered 0 = start, then per function)."""
    src = parse(text)
    for f, fn in src.functions.items():  # bodies are closed: inlining cannot capture names
        _check_defined(f, fn.body, fn.params)
    dec = decomposed_functions(src)
    bodies = inline(src, dec)
    for f in bodies:
        bodies[f] = _tail_calls(f, src.functions[f].params, bodies[f])
    counter = itertools.count(1)
    order = sorted(bodies, key=lambda g: (g != "main", g))
    decomposed = {}
    for f in order:
        _check_defined(f, bodies[f], src.functions[f].params)
        d = Decomposer(_kind(dec), counter)
        decomposed[f] = d.decompose(bodies[f])
    # locals that a single block uses live in that block's registers; the rest
    # (and parameters and call results) in the frame
    frames, slots, block_regs = {}, {}, {}
    for f in order:
        params = src.functions[f].params
        entry, blocks = decomposed[f]
        users = {}
        for idx, items in blocks.items():
            for v in _block_names(items, set()):
                users.setdefault(v, set()).add(idx)
        results = {s[1] for s in _walk(bodies[f]) if s[0] == "call"}
        assigned = [v for v in _assigned(bodies[f]) if v not in params]
        in_regs = set()
        for idx in blocks:
            mine = [v for v in assigned if users.get(v) == {idx} and v not in results][:REG_LOCALS]
            block_regs[idx] = {v: N_REGS - 1 - i for i, v in enumerate(mine)}
            in_regs.update(mine)
        names = params + [v for v in assigned if v not in in_regs]
        if any(s[0] == "tailcall" for s in _walk(bodies[f])) and len(params) > MAX_TAIL_ARGS:
            names += [f"$tail{i}" for i in range(len(params))]  # staging for a long tail call
        slots[f] = {v: 2 + i for i, v in enumerate(names)}
        frames[f] = 2 + len(names)
    # final numbering: 0 = start block, then each function's blocks, entry first
    block_of, names = {}, ["start"]
    for f in order:
        entry, blocks = decomposed[f]
        for idx in [entry] + sorted(i for i in blocks if i != entry):
            block_of[idx] = len(names)
            names.append(f"{f}:{idx}")
    if len(names) > MAX_BLOCKS:
        raise CompileError(f"{len(names)} blocks; at most {MAX_BLOCKS}")
    entries = {f: block_of[decomposed[f][0]] for f in order}
    gen = _Gen(src, frames, slots, entries, block_of)
    code, starts = [], []
    # start block: main's frame with return block b_stop; its return value
    # location is its own slot 1
    fm = frames["main"]
    start = [["FRAME", 0, 0, 0, 0], ["CALLFRAME", 0, 0, 0, fm], ["IMM", 0, 0, 0, STOP], ["STN", 0, 0, 0, 0],
             ["IMM", 0, 0, 0, 1], ["STN", 0, 0, 0, 1], ["PUSH", 0, 0, 0, fm], ["GOTO", 0, 0, 0, entries["main"]],
             ["FAULT", 0, 0, 0, 0]]
    blocks_code = [start]
    for f in order:
        entry, blocks = decomposed[f]
        for idx in [entry] + sorted(i for i in blocks if i != entry):
            out = [["FRAME", 0, 0, 0, frames[f]]]
            gen.regs = block_regs[idx]
            gen.limit = N_REGS - len(gen.regs)
            gen.tstmts(blocks[idx], f, out)
            out.append(["FAULT", 0, 0, 0, 0])
            blocks_code.append(out)
    for blk in blocks_code:
        base = len(code)
        starts.append(base)
        for ins in blk:
            op, x, y, z, imm = ins
            if op in ("JZ", "JMP"):
                imm = base + imm
            code.append(_enc(op, x, y, z, imm))
    starts.append(len(code))
    if max(frames.values()) > stack_words:
        raise CompileError(f"a frame of {max(frames.values())} words exceeds the stack of {stack_words}")
    data = [v for name in gen.arrays for v in src.data[name]]
    astart = np.cumsum([0] + [len(src.data[n]) for n in gen.arrays]).astype(np.uint32)
    return ProgramImage(code=np.array(code, dtype=np.uint64), block_start=np.array(starts, dtype=np.uint32),
                        consts=np.array(gen.consts or [0.0], dtype=np.float64),
                        data=np.array(data, dtype=np.float64), array_start=astart,
                        stack_words=int(stack_words), block_names=names, frames=frames, entry=entries)


def decode_op(word: int):
    """(opcode name, x, y, z, signed immediate) of one instruction word."""
    inv = {v: name for name, v in OPS.items()}
    imm = word >> 32
    if imm >= 1 << 31:
        imm -= 1 << 32
    return inv.get(word & 255, word & 255), (word >> 8) & 255, (word >> 16) & 255, (word >> 24) & 255, imm


def disassemble(img: ProgramImage) -> str:
    inv = {v: k for k, v in OPS.items()}
    lines = []
    for b in range(img.n_blocks):
        lines.append(f"block {b} ({img.block_names[b] if b < len(img.block_names) else ''}):")
        for pc in range(int(img.block_start[b]), int(img.block_start[b + 1])):
            w = int(img.code[pc])
            op, x, y, z, imm = w & 255, (w >> 8) & 255, (w >> 16) & 255, (w >> 24) & 255, w >> 32
            if imm >= 1 << 31:
                imm -= 1 << 32
            lines.append(f"  {pc:4d} {inv.get(op, op):9s} {x:2d} {y:2d} {z:2d} {imm}")
    return "\n".join(lines)
