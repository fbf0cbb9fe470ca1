"""Sequential CPU simulator of the program bytecode (test tool).

Executes a compiled program image one particle at a time with the instruction
semantics documented in include/pcfgsmc.h, and drives Algorithm 1 over it with
the oracle's resampling. It exists so the CPU tests can check the compiler
(Algorithm 2, frames, code generation) against the source-level oracle
without a GPU; the GPU tests compare the library's interpreter with the
oracle directly.
"""
from __future__ import annotations

import math

import numpy as np

from oracle import oracle as O
from oracle import ppl_oracle as PO

STOP = 255
BUDGET = 1 << 20
NAMES = {1: "FRAME", 2: "CONST", 3: "IMM", 4: "MOV", 5: "LDF", 6: "STF", 7: "ADD", 8: "SUB", 9: "MUL",
         10: "DIV", 11: "LT", 12: "LE", 13: "EQ", 14: "NE", 15: "NEG", 16: "NOT", 17: "LOG", 18: "EXP",
         19: "SQRT", 20: "FLOOR", 21: "DATA", 22: "LEN", 23: "SAMPLE", 24: "OBSERVE", 25: "WEIGHT",
         26: "JZ", 27: "JMP", 28: "CALLFRAME", 29: "STN", 30: "ADDR", 31: "PUSH", 32: "STRET", 33: "GOTO",
         34: "CKPT", 35: "JRET", 36: "FAULT"}
OBS_NAMES = {0: "uniform", 1: "normal", 2: "exponential", 5: "bernoulli", 6: "poisson", 7: "binomial"}


def decode(w):
    w = int(w)
    imm = w >> 32
    return NAMES[w & 255], (w >> 8) & 255, (w >> 16) & 255, (w >> 24) & 255, imm


class Fault(Exception):
    pass


def run_blocks(img, code, p, seed, slot, rnd):
    """p = [blk, sp, stack(list), lw]; runs to a checkpoint or b_stop. Returns block steps."""
    blk, sp, st, lw = p
    k = 0
    reg = [0.0] * 16
    steps = 0
    executed = 0
    f64 = np.float64
    try:
        while blk != STOP:
            steps += 1
            pc = int(img.block_start[blk])
            fp = 0
            opened = 0
            while True:
                op, x, y, z, imm = code[pc]
                pc += 1
                executed += 1
                if executed > BUDGET:
                    raise Fault()
                if op == "FRAME":
                    if sp < imm:
                        raise Fault()
                    fp = sp - imm
                elif op == "CONST":
                    reg[x] = float(img.consts[imm])
                elif op == "IMM":
                    reg[x] = float(imm - (1 << 32) if imm >= 1 << 31 else imm)
                elif op == "MOV":
                    reg[x] = reg[y]
                elif op == "LDF":
                    assert st[fp + imm] is not None, "read of an unwritten stack word"
                    reg[x] = st[fp + imm]
                elif op == "STF":
                    st[fp + imm] = reg[x]
                elif op in ("ADD", "SUB", "MUL", "DIV"):
                    with np.errstate(all="ignore"):
                        a, b = f64(reg[y]), f64(reg[z])
                        reg[x] = float({"ADD": a + b, "SUB": a - b, "MUL": a * b, "DIV": a / b}[op])
                elif op in ("LT", "LE", "EQ", "NE"):
                    a, b = reg[y], reg[z]
                    reg[x] = 1.0 if {"LT": a < b, "LE": a <= b, "EQ": a == b, "NE": a != b}[op] else 0.0
                elif op == "NEG":
                    reg[x] = -reg[y]
                elif op == "NOT":
                    reg[x] = 1.0 if reg[y] == 0.0 else 0.0
                elif op == "LOG":
                    reg[x] = O.log(reg[y])
                elif op == "EXP":
                    reg[x] = O.exp(reg[y])
                elif op == "SQRT":
                    with np.errstate(all="ignore"):
                        reg[x] = float(np.sqrt(f64(reg[y])))
                elif op == "FLOOR":
                    reg[x] = float(np.floor(f64(reg[y])))
                elif op == "DATA":
                    a0, a1 = int(img.array_start[imm]), int(img.array_start[imm + 1])
                    v = reg[y]
                    if not (v >= 0.0 and v < a1 - a0 and v == math.floor(v)):
                        raise Fault()
                    reg[x] = float(img.data[a0 + int(v)])
                elif op == "LEN":
                    reg[x] = float(int(img.array_start[imm + 1]) - int(img.array_start[imm]))
                elif op == "SAMPLE":
                    v, k, fault = O.draw(imm, reg[y], reg[z], seed, slot, rnd, k)
                    if fault:
                        raise Fault()
                    reg[x] = v
                elif op == "OBSERVE":
                    name = OBS_NAMES[imm]
                    args = [reg[y]] if name in ("exponential", "bernoulli", "poisson") else [reg[y], reg[z]]
                    try:
                        lw = lw + PO.observe_logpdf(name, args, reg[x])
                    except PO.Fault:
                        raise Fault()
                elif op == "WEIGHT":
                    lw = lw + reg[x]
                elif op == "JZ":
                    if reg[x] == 0.0:
                        pc = imm
                elif op == "JMP":
                    pc = imm
                elif op == "CALLFRAME":
                    if imm > img.stack_words - sp:
                        raise Fault()
                    opened = imm
                elif op == "STN":
                    st[sp + imm] = reg[x]
                elif op == "ADDR":
                    reg[x] = float(fp + imm)
                elif op == "PUSH":
                    assert imm == opened
                    sp += imm
                elif op == "STRET":
                    loc = st[fp + 1]
                    if not (loc >= 0 and loc < sp and loc == math.floor(loc)):
                        raise Fault()
                    st[int(loc)] = reg[x]
                elif op in ("GOTO", "CKPT", "JRET"):
                    nxt = imm
                    if op == "JRET":
                        ra = st[fp]
                        if ra == STOP:
                            nxt = STOP
                        elif ra >= 0 and ra < img.n_blocks and ra == math.floor(ra):
                            nxt = int(ra)
                        else:
                            raise Fault()
                        sp -= imm
                    blk = nxt
                    if op == "CKPT" and blk != STOP:
                        p[:] = [blk, sp, st, lw]
                        return steps
                    break
                else:
                    raise Fault()
        p[:] = [STOP, sp, st, lw]
        return steps
    except Fault:
        p[:] = [STOP, 0, st, -math.inf]
        return steps


class SimRun:
    """Algorithm 1 over the simulated bytecode (same resampling as the oracle)."""

    def __init__(self, img, n, seed, ess_threshold=0.0):
        self.img, self.n, self.seed = img, int(n), int(seed)
        self.code = [decode(w) for w in img.code]
        self.ess = float(ess_threshold)
        # None marks a stack word no instruction has written (its device value is undefined)
        self.p = [[0, 0, [None] * img.stack_words, 0.0] for _ in range(self.n)]
        self.round, self.log_z, self.status, self.block_steps = 0, 0.0, O.OK, 0
        self.anc = np.arange(self.n, dtype=np.uint32)

    def lw(self):
        return np.array([q[3] for q in self.p])

    def step(self):
        for j, q in enumerate(self.p):
            if q[0] != STOP:
                self.block_steps += run_blocks(self.img, self.code, q, self.seed, j, self.round)

    def resample(self):
        lw = self.lw()
        active = any(q[0] != STOP for q in self.p)
        resample = True
        if active and self.ess > 0.0:
            resample = O.ess_resamples(lw, self.ess) == 1
        st, anc, inc, _ = O.systematic(lw, self.seed, self.round)
        if st == O.DEGENERATE:
            self.log_z, self.status = -math.inf, st
            return st
        if st != O.OK:
            self.status = st
            return st
        if not active:
            self.log_z += inc
            self.status = O.FINISHED
            return self.status
        if not resample:
            self.anc = np.arange(self.n, dtype=np.uint32)
            self.round += 1
            return O.OK
        self.log_z += inc
        self.anc = anc
        # live-prefix copy: words beyond sp are not carried
        self.p = [[self.p[a][0], self.p[a][1], self.p[a][2][:self.p[a][1]] + [None] * (self.img.stack_words - self.p[a][1]),
                   0.0] for a in anc]
        self.round += 1
        return O.OK

    def run_to_end(self, max_rounds=100000):
        for _ in range(max_rounds):
            if self.status != O.OK:
                break
            self.step()
            self.resample()
        return self.status
