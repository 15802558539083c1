"""Write tests/golden/c3_512_samples.npz: the FP64 oracle on the C3 cloud at 512^3.

Workload: the C3 cloud (100,000 points on a superellipsoid with noisy
normals, seed 2) on a 512^3 grid, sigma 2 cells, reading B; the loss
gradient G is psr_synth.loss_gradient(512, 512). Stored: chi at 8192 voxels
drawn by PCG64(513), max|chi| over the whole grid, mu, c and s, and
dL/dpoints and dL/dnormals at 4096 points drawn by PCG64(514) with the L2
norms of the full gradient arrays. The full arrays (512 MB each) are not
kept: the GPU test compares these samples.

Run: python tests/golden/make_c3_512.py   (about 6 minutes, 36 GB of memory)
"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
import psr_synth as S  # noqa: E402

RES, SIGMA = 512, 2.0
N_VOX, N_PTS = 8192, 4096


def main():
    sh = S.config_c3()
    chi, aux = oracle.forward(sh.points, sh.normals, RES, SIGMA)
    assert aux["status"] == "ok"
    vox = S.rng_for(513).choice(RES ** 3, N_VOX, replace=False).astype(np.int64)
    chi_s = chi.reshape(-1)[vox].copy()
    chi_max = float(np.abs(chi).max())
    del chi
    G = S.loss_gradient(RES, 512)
    dc, dn = oracle.backward(aux, G)
    pts = S.rng_for(514).choice(sh.P, N_PTS, replace=False).astype(np.int64)
    np.savez_compressed(os.path.join(HERE, "c3_512_samples.npz"),
                        vox=vox, chi=chi_s, chi_max=chi_max, mu=aux["mu"], cscale=aux["cscale"], scale=aux["s"],
                        pts=pts, dpoints=dc[pts], dnormals=dn[pts],
                        dpoints_norm=float(np.linalg.norm(dc)), dnormals_norm=float(np.linalg.norm(dn)))
    print("mu", aux["mu"], "c", aux["cscale"], "max|chi|", chi_max)


if __name__ == "__main__":
    main()
