"""Oracle for applications given as C source (test infrastructure only).

The reference result of a C program is the program itself, run serially: the
whole unmodified source -- every loop nest in program order, the iterated
blocks as the plain for loops they are -- compiled with g++ at -O2 and
``-ffp-contract=off`` (every float expression evaluated as written) and run
once on the set-up content of its arrays.  Offloading loops must not change
what a program computes (Sec. 3.3, Sec. 4), so every offload pattern's result
is compared with this run.

The source is read here on its own terms (independently of the library's C
front end): ``#define NAME <int>`` lines, array declarations
``float|double|bf16 NAME[d]...;`` with an optional ``// ofl: output
setup=sin mode=M`` annotation (zero set-up otherwise), ``#pragma`` lines
(ignored), and the statements, which become the body of one function.  The
arrays are the caller's numpy buffers.  Supported calls: the C math library
and ``bf16(x)`` (round a float to the nearest bfloat16, ties to even); the
counter-based ``u01`` and the sequential ``lcg01`` are not defined here (a
program using them is checked through the nest-by-nest oracle in run.py).
"""
import ctypes
import hashlib
import os
import re
import subprocess

import numpy as np

from . import cnests as C

_HERE = os.path.dirname(os.path.abspath(__file__))
_CACHE = os.path.join(_HERE, "_cprog")
CXXFLAGS = ["-O2", "-std=c++17", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared", "-w"]

_DEFINE = re.compile(r"\s*#define\s+([A-Za-z_]\w*)\s+(-?\d+)\s*$")
_ARRAY = re.compile(r"\s*(float|double|bf16)\s+([A-Za-z_]\w*)((?:\s*\[[^\]]+\])+)\s*;\s*(?://\s*ofl:(.*))?$")
_NP = {"float": np.float32, "double": np.float64, "bf16": np.uint16}

_PRELUDE = """#include <cmath>
#include <cstdint>
#include <cstring>
#include <math.h>
#include <stdlib.h>

namespace {
// bfloat16 held as its 16-bit pattern; bf16(x): round to nearest, ties to
// even (a NaN stays a quiet NaN); used as a float it is widened exactly
struct bf16 {
    uint16_t h;
    bf16() = default;
    bf16(float x) {
        uint32_t u;
        std::memcpy(&u, &x, sizeof u);
        const uint32_t exp_all = 0x7F800000u, man = 0x007FFFFFu;
        if ((u & exp_all) == exp_all && (u & man) != 0) {
            h = (uint16_t)((u >> 16) | 0x0040u);
        } else {
            const uint32_t lsb = (u >> 16) & 1u;
            h = (uint16_t)((u + 0x00007FFFu + lsb) >> 16);
        }
    }
    operator float() const {
        uint32_t u = (uint32_t)h << 16;
        float x;
        std::memcpy(&x, &u, sizeof x);
        return x;
    }
};
}  // namespace
"""


class Program:
    """A C program split into parameters, arrays and statements."""

    def __init__(self, src):
        self.params, self.arrays, body = {}, [], []
        for line in src.splitlines():
            m = _DEFINE.match(line)
            if m:
                self.params[m.group(1)] = int(m.group(2))
                continue
            m = _ARRAY.match(line)
            if m:
                dims = [d.strip() for d in re.findall(r"\[([^\]]+)\]", m.group(3))]
                opts = (m.group(4) or "").split()
                setup = next((o.split("=", 1)[1] for o in opts if o.startswith("setup=")), "zero")
                mode = next((o.split("=", 1)[1] for o in opts if o.startswith("mode=")), "1")
                self.arrays.append({"type": m.group(1), "name": m.group(2), "dims": dims, "setup": setup,
                                    "mode": mode, "output": "output" in opts})
                continue
            if line.lstrip().startswith("#"):
                continue
            body.append(line)
        self.body = "\n".join(body)
        for bad in ("u01", "lcg01"):
            if re.search(r"\b%s\s*\(" % bad, self.body):
                raise ValueError("%s() has no definition in the compiled-program oracle" % bad)

    def value(self, text):
        return int(eval(text, {"__builtins__": {}}, dict(self.params)))

    def shape(self, a):
        return tuple(self.value(d) for d in a["dims"])

    def unit(self):
        out = [_PRELUDE]
        out += ["#define %s %d" % kv for kv in self.params.items()]
        out.append('extern "C" void oracle_program(void **arr) {')
        for i, a in enumerate(self.arrays):
            ty = a["type"]
            if len(a["dims"]) == 1:
                out.append("    %s *%s = (%s *)arr[%d];" % (ty, a["name"], ty, i))
            else:
                tail = "".join("[%s]" % d for d in a["dims"][1:])
                out.append("    %s (*%s)%s = (%s (*)%s)arr[%d];" % (ty, a["name"], tail, ty, tail, i))
        out.append(self.body)
        out.append("}")
        return "\n".join(out) + "\n"

    def setup(self):
        """Set-up content: zeros, or the sine field of the oracle's nests."""
        bufs = {}
        for a in self.arrays:
            shp = self.shape(a)
            if a["setup"] == "sin":
                bufs[a["name"]] = C.sin_field(*shp, self.value(a["mode"]))
            else:
                bufs[a["name"]] = np.zeros(shp, _NP[a["type"]])
        return bufs


def build(prog):
    unit = prog.unit()
    key = hashlib.sha256(unit.encode()).hexdigest()[:16]
    so = os.path.join(_CACHE, "prog_%s.so" % key)
    if not os.path.exists(so):
        os.makedirs(_CACHE, exist_ok=True)
        src = os.path.join(_CACHE, "prog_%s.cpp" % key)
        with open(src, "w") as f:
            f.write(unit)
        tmp = so + ".tmp%d" % os.getpid()
        subprocess.check_call(["g++"] + CXXFLAGS + [src, "-o", tmp, "-lm"])
        os.replace(tmp, so)
    return so


def run_program(src):
    """Serial run of the whole program: {array name: numpy array}."""
    prog = Program(src)
    lib = ctypes.CDLL(build(prog))
    bufs = prog.setup()
    ptrs = (ctypes.c_void_p * len(prog.arrays))(*[bufs[a["name"]].ctypes.data for a in prog.arrays])
    lib.oracle_program.restype = None
    lib.oracle_program.argtypes = [ctypes.POINTER(ctypes.c_void_p)]
    lib.oracle_program(ptrs)
    return bufs
