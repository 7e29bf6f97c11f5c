"""Write the analytic force/torque map of the metallo-dielectric Janus cylinder
at a / lambda = 1 on a subgrid of the paper's design map.

The paper's map (Sec. IV.A, Fig. HS75_Map (a)-(c), LBM; (d)-(f), its error
against the analytic solution) spans phi0 = 0 .. 2 pi in steps of pi / 90
and eps_r1 = 1 .. 5 in steps of 0.04.  Here every other point of each axis:
phi0 = j pi / 45 (j = 0 .. 90) and eps_r1 = 1 + 0.08 i (i = 0 .. 50), from
oracle/analytic.py only (Eqs. integral equation, constants_Bm_Dm,
coefficients, U, V, Torque), Richardson-extrapolated over N = 257, 513, 1025
(agrees with N = 513, 1025, 2049 to 1e-5 at the convergence point of
Sec. IV.A.2).  The mirror rule (F~x, F~y, M~z)(phi0) = (F~x, -F~y, -M~z)(pi - phi0)
halves the work.  Run from the repository root:

    python tests/golden/make_map_analytic.py
"""
import json
import math
import os
import sys
from multiprocessing import Pool

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import analytic as A  # noqa: E402

NPHI, NEPS = 91, 51


def eps_of(i):
    return round(1.0 + 0.08 * i, 10)


def one(args):
    i, j = args
    q, _, _ = A.mdjc_forces_extrapolated(2 * math.pi, eps_of(i), j * math.pi / 45, N=257)
    return i, j, [float(v) for v in q]


def main():
    # representative of j under phi0 -> pi - phi0 (mod 2 pi): index (45 - j) mod 90
    todo = []
    for i in range(NEPS):
        for j in range(NPHI):
            m = (45 - j) % 90
            if j <= m or j == 90:
                todo.append((i, j))
    with Pool(int(os.environ.get("MAP_WORKERS", os.cpu_count() or 1))) as pool:
        got = {}
        for k, (i, j, q) in enumerate(pool.imap_unordered(one, todo, chunksize=8)):
            got[(i, j)] = q
            if k % 200 == 0:
                print(f"{k}/{len(todo)}", flush=True)
    fx = [[0.0] * NPHI for _ in range(NEPS)]
    fy = [[0.0] * NPHI for _ in range(NEPS)]
    tz = [[0.0] * NPHI for _ in range(NEPS)]
    for i in range(NEPS):
        for j in range(NPHI):
            if (i, j) in got:
                q, s = got[(i, j)], 1.0
            elif j == 90:
                q, s = got[(i, 0)], 1.0
            else:
                q, s = got[(i, (45 - j) % 90)], -1.0
            fx[i][j] = round(q[0], 7)
            fy[i][j] = round(s * q[1], 7)
            tz[i][j] = round(s * q[2], 7)
    out = {"note": "analytic MDJC (F~x, F~y, M~z) at a/lambda = 1; rows eps_r1 = 1 + 0.08 i, columns "
                   "phi0 = j pi/45; Richardson over N = 257, 513, 1025; written by tests/golden/make_map_analytic.py",
           "eps1": [eps_of(i) for i in range(NEPS)], "phi0": [j * math.pi / 45 for j in range(NPHI)],
           "fx": fx, "fy": fy, "tz": tz}
    with open(os.path.join(ROOT, "tests", "golden", "mdjc_map_analytic.json"), "w") as f:
        json.dump(out, f, separators=(",", ":"))


if __name__ == "__main__":
    main()
