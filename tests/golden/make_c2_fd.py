"""Write tests/golden/c2_fd.json: FP64 central finite differences of the C2 loss.

Workload (128^3, sigma 2, seed 1): 20,000 points on a torus U sphere, inputs
jittered by N(0, 0.002^2); target chi_t is the forward on the clean points;
loss L = mean((chi - chi_t)^2). For 64 random position coordinates and 64
random normal coordinates, dL/dx is estimated by (L(x+h) - L(x-h)) / 2h with
h = 1e-4 on the FP64 oracle only. Position coordinates whose cell fraction
lies within 2 r h of a cell face are skipped (the trilinear weights have a
kink there). The analytic oracle gradient at the same coordinates and the
infinity norms of the full oracle gradients are stored beside them.

Run: python tests/golden/make_c2_fd.py   (uses all cores, about a minute)
"""
import json
import os
import sys
from multiprocessing import Pool

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
import psr_synth as S  # noqa: E402

H_STEP = 1e-4
N_COORD = 64

_state = {}


def _init():
    sh = S.config_c2()
    chi_t, _ = oracle.forward(sh.points_clean, sh.normals_clean, sh.res, sh.sigma)
    _state.update(sh=sh, chi_t=chi_t)


def _loss(c, n):
    sh = _state["sh"]
    chi, _ = oracle.forward(c, n, sh.res, sh.sigma)
    return float(((chi - _state["chi_t"]) ** 2).mean())


def _fd(task):
    which, i, a = task
    sh = _state["sh"]
    c = sh.points.astype(np.float64)
    n = sh.normals.astype(np.float64)
    tgt = c if which == "points" else n
    tgt[i, a] += H_STEP
    lp = _loss(c, n)
    tgt[i, a] -= 2 * H_STEP
    lm = _loss(c, n)
    return (lp - lm) / (2 * H_STEP)


def main():
    sh = S.config_c2()
    r = sh.res
    chi_t, _ = oracle.forward(sh.points_clean, sh.normals_clean, r, sh.sigma)
    chi, aux = oracle.forward(sh.points, sh.normals, r, sh.sigma)
    G = 2.0 * (chi - chi_t) / chi.size
    dc, dn = oracle.backward(aux, G)
    rng = np.random.Generator(np.random.PCG64(12345))
    tasks = []
    while len([t for t in tasks if t[0] == "points"]) < N_COORD:
        i, a = int(rng.integers(0, sh.P)), int(rng.integers(0, 3))
        frac = (r * float(sh.points[i, a])) % 1.0
        if 2 * r * H_STEP < frac < 1 - 2 * r * H_STEP:
            tasks.append(("points", i, a))
    for _ in range(N_COORD):
        tasks.append(("normals", int(rng.integers(0, sh.P)), int(rng.integers(0, 3))))
    with Pool(min(8, os.cpu_count() or 1), initializer=_init) as pool:
        fds = pool.map(_fd, tasks)
    out = dict(
        citation="Finite-difference check of dL/dpoints, dL/dnormals on the FP64 oracle (main Sec. 3.1: the "
                 "solver is differentiable w.r.t. the oriented points). Written by tests/golden/make_c2_fd.py.",
        config="C2: 128^3, sigma 2, seed 1, 20000 points, torus U sphere, jitter N(0,0.002^2), "
               "loss = mean((chi - chi_t)^2), chi_t from clean points",
        h=H_STEP,
        grad_inf_points=float(np.abs(dc).max()), grad_inf_normals=float(np.abs(dn).max()),
        entries=[dict(which=w, i=i, a=a, fd=float(f),
                      oracle=float((dc if w == "points" else dn)[i, a])) for (w, i, a), f in zip(tasks, fds)],
    )
    with open(os.path.join(HERE, "c2_fd.json"), "w") as fh:
        json.dump(out, fh, indent=1)
    worst = max(abs(e["fd"] - e["oracle"]) / max(abs(e["fd"]), 1e-3 * (out["grad_inf_points"] if e["which"] == "points"
                                                                         else out["grad_inf_normals"]))
                for e in out["entries"])
    print("written; worst oracle-vs-FD relative deviation", worst)


if __name__ == "__main__":
    main()
