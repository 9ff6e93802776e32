"""The OpenMP build of the oracle (liboracle_omp.so, the benchmark's
multi-core CPU timing) against the plain build: the same source with its
per-row loops on several threads, so every result must be the same bit for
bit (reductions and scatter-adds stay serial)."""
import json
import os
import subprocess
import sys

import numpy as np

import synth
from oracle import oracle as orc

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

CHILD = r"""
import json, sys
import numpy as np
sys.path.insert(0, ROOT)
import synth
from oracle import oracle as orc
rec = synth.recipe("c3", n=20)
rec.options.precision = synth.FP64
ks, p0 = rec.ks(), rec.p0()
th = orc.theta(rec.problem, p0)
F = orc.residual(rec.problem, ks, p0, th)
J = orc.jacobian(rec.problem, ks, p0)
M = orc.auxiliary(rec.problem, ks, p0)
amg = orc.AMG(rec.options, M)
z = amg.apply(F)
x, its = orc.gmres(J, -F, amg, 30, 1e-8, 200)[:2]
s = orc.Solver(rec.problem, rec.options, ks)
p = p0.copy()
st = s.step(p)
print(json.dumps({"theta": th.tobytes().hex(), "F": F.tobytes().hex(), "J": J.data.tobytes().hex(),
                  "Jp": J.indptr.tobytes().hex(), "M": M.data.tobytes().hex(), "z": z.tobytes().hex(),
                  "x": x.tobytes().hex(), "its": int(its), "p": p.tobytes().hex(),
                  "newton": st["newton_its"], "gmres": st["gmres_its"]}))
""".replace("ROOT", repr(ROOT))


def run(omp):
    env = dict(os.environ, OMP_NUM_THREADS="4")
    if omp:
        env["RICH_ORACLE_OMP"] = "1"
    else:
        env.pop("RICH_ORACLE_OMP", None)
    r = subprocess.run([sys.executable, "-c", CHILD], env=env, capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr
    return json.loads(r.stdout.strip().splitlines()[-1])


def test_openmp_build_bitwise():
    orc.build()
    assert os.path.exists(orc.OMP_LIB_PATH)
    a, b = run(False), run(True)
    for k in a:
        assert a[k] == b[k], k
