"""Launch-shape tuning for libtik.

Times the candidate launch shapes of the two products over A on problems of
the given shapes (tik_tune: a fixed number of batched FP64 LSQR iterations per
candidate) and writes the table the library reads on first use
(``tuning.txt`` beside libtik.so, unless --out says otherwise).

    python -m paper_2203_07329_amd.tune [--out PATH] [--iters K] [SPEC ...]

A SPEC names one shape class by an example of it:

    tall:MxN:N32            one tall FP64 problem, 32 lambdas
    wide:MxN:f32:N32        one wide problem stored in FP32
    ragged:P:MLO-MHIxNLO-NHI:f32:N8   P tall problems, sizes uniform in the ranges
    lowrank:MxN:f32:N16:s1842          the low-rank route with sketch size s

Values do not matter to the timing (every candidate runs the same number of
iterations), so the matrices are Gaussian, drawn on the device from a fixed
seed.  With no SPEC the classes of the library's benchmark workloads are tuned.
"""

import argparse
import os
import re
import sys

import numpy as np
import torch

from . import tik

DEFAULT_SPECS = [
    "tall:200000x2000:N32",
    "wide:2000x200000:f32:N32",
    "ragged:256:5000-50000x100-1000:f32:N8",
    "lowrank:100000x10000:f32:N16:s1842",
    "tall:50000x1000:N16",
]


def parse(spec: str) -> dict:
    parts = spec.split(":")
    kind = parts[0]
    if kind not in ("tall", "wide", "ragged", "lowrank"):
        raise ValueError("unknown kind in " + spec)
    d = {"kind": kind, "f32": False, "N": 32, "s": None, "P": 1}
    rest = parts[1:]
    if kind == "ragged":
        d["P"] = int(rest[0])
        m = re.fullmatch(r"(\d+)-(\d+)x(\d+)-(\d+)", rest[1])
        if not m:
            raise ValueError("ragged sizes must read MLO-MHIxNLO-NHI: " + spec)
        d["mr"] = (int(m[1]), int(m[2]))
        d["nr"] = (int(m[3]), int(m[4]))
        rest = rest[2:]
    else:
        m = re.fullmatch(r"(\d+)x(\d+)", rest[0])
        if not m:
            raise ValueError("size must read MxN: " + spec)
        d["m"], d["n"] = int(m[1]), int(m[2])
        rest = rest[1:]
    for r in rest:
        if r == "f32":
            d["f32"] = True
        elif r.startswith("N"):
            d["N"] = int(r[1:])
        elif r.startswith("s"):
            d["s"] = int(r[1:])
        else:
            raise ValueError("unknown field %r in %s" % (r, spec))
    return d


def problems(d: dict, gen: torch.Generator):
    dt = torch.float32 if d["f32"] else torch.float64
    if d["kind"] == "ragged":
        rng = np.random.default_rng(0)
        ms = rng.integers(d["mr"][0], d["mr"][1] + 1, size=d["P"])
        ns = np.minimum(rng.integers(d["nr"][0], d["nr"][1] + 1, size=d["P"]), ms)
        shapes = list(zip(ms.tolist(), ns.tolist()))
    else:
        shapes = [(d["m"], d["n"])]
    At = [torch.randn((n, m), dtype=dt, device="cuda", generator=gen) for m, n in shapes]
    b = [torch.randn(m, dtype=torch.float64, device="cuda", generator=gen) for m, _ in shapes]
    return tik.Problems(At, b), shapes


def tune_spec(spec: str, iters: int) -> str:
    d = parse(spec)
    gen = torch.Generator(device="cuda")
    gen.manual_seed(1)
    probs, shapes = problems(d, gen)
    lams = np.logspace(-6, -1, d["N"])
    if d["kind"] == "lowrank":
        s = d["s"] or 2 * min(shapes[0])
        pc = tik.precond(tik.sketch(probs, tik.SRHT, [s], 0), lams, tik.ROUTE_LOWRANK)
    elif d["kind"] == "wide":
        pc = tik.precond(tik.sketch(probs, tik.GAUSS, [d["s"] or 4 * shapes[0][0]], 0), lams)
    else:
        embed = tik.GAUSS if d["kind"] == "ragged" else tik.SRHT
        s = [d["s"] or min(4 * n, m) for m, n in shapes]
        pc = tik.precond(tik.sketch(probs, embed, s, 0), lams)
    best, best_ms, default_ms = tik.tune(probs, pc, iters)
    return ("%-40s rows %3d cols %3d blocks %4d: %8.3f ms per %d iterations (default shape %8.3f ms)"
            % (spec, best[0], best[1], best[2], best_ms, iters, default_ms))


def main(argv=None) -> int:
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("specs", nargs="*", default=DEFAULT_SPECS)
    ap.add_argument("--out", default=os.path.join(os.path.dirname(os.path.abspath(tik.__file__)),
                                                  "tuning.txt"))
    ap.add_argument("--iters", type=int, default=20)
    a = ap.parse_args(argv)
    if not torch.cuda.is_available():
        print("tune: no GPU", file=sys.stderr)
        return 1
    for spec in a.specs:
        print(tune_spec(spec, a.iters), flush=True)
        torch.cuda.empty_cache()
    tik.tune_save(a.out)
    print("wrote", a.out, flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
