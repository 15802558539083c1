"""Write the GPU's error against the FP64 oracle for every benchmark workload
to a JSON summary (run on a GPU host; the pytest parity tests are the gate,
this file is the record of the numbers they check).

    python tests/parity_summary.py OUT.json

Workloads: the 32^3 sphere (forward), the 128^3 torus + sphere with its
finite-difference entries, the same with half the points outliers, the 256^3
superellipsoid, the 256^3 cloud on 512^3 against stored oracle samples, the
thin closed plate at 64^3 and 128^3, each of the 64 shapes of the batched
workload solved in one batch, and the slab-decomposed forward (256^3 against
the oracle, 512^3 against the stored samples, one Fourier mode at 1024^3
against its closed form). Metrics: e_chi = max|chi_gpu -
chi_ref| / max|chi_ref|, e_dpoints and e_dnormals = relative L2 error; bars
1e-5 and 1e-4. Each side forms its own loss gradient (G = 2 (chi - chi_t) / N
for the benchmark losses, G = 2 chi / N for the batch).
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
sys.path.insert(0, ROOT)
sys.path.insert(0, HERE)

import oracle  # noqa: E402
import psr_synth as S  # noqa: E402
from gpu_common import host, l2_rel, max_rel, to_dev, torch  # noqa: E402


def say(msg):
    print(f"[parity] {msg}", flush=True)


def run_pair(F, sh, dev, with_target=True):
    """GPU and oracle forward + backward of one workload; returns the errors."""
    pts, nrm = to_dev(sh.points, dev), to_dev(sh.normals, dev)
    chi, saved = F.forward(pts, nrm, sh.res, sh.sigma)
    ref, aux = oracle.forward(sh.points, sh.normals, sh.res, sh.sigma)
    out = {"res": sh.res, "npoints": sh.P, "status": F.status(saved), "e_chi": max_rel(host(chi), ref)}
    if not with_target:
        return out
    if sh.points_clean is not None:
        chi_t, _ = F.forward(to_dev(sh.points_clean, dev), to_dev(sh.normals_clean, dev), sh.res, sh.sigma)
        ref_t, _ = oracle.forward(sh.points_clean, sh.normals_clean, sh.res, sh.sigma)
        G, G_r = 2.0 * (chi - chi_t) / chi.numel(), 2.0 * (ref - ref_t) / ref.size
    else:
        G, G_r = to_dev(S.loss_gradient(sh.res, sh.res), dev), S.loss_gradient(sh.res, sh.res).astype(np.float64)
    dp, dn = F.backward(chi, saved, G.contiguous(), sh.P, sh.res, sh.sigma)
    dc_r, dn_r = oracle.backward(aux, G_r)
    out.update(e_dpoints=l2_rel(host(dp), dc_r), e_dnormals=l2_rel(host(dn), dn_r))
    return out


def fd_entries(dp, dn):
    fd = json.load(open(os.path.join(HERE, "golden", "c2_fd.json")))
    out = {}
    for kind, g_all in (("points", dp), ("normals", dn)):
        ent = [e for e in fd["entries"] if e["which"] == kind]
        g = np.array([g_all[e["i"], e["a"]] for e in ent])
        f = np.array([e["fd"] for e in ent])
        inf = fd["grad_inf_" + kind]
        out[kind] = {"n": len(ent), "l2_rel": float(np.linalg.norm(g - f) / np.linalg.norm(f)),
                     "worst_entry": float(np.max(np.abs(g - f) / np.maximum(np.abs(f), 1e-3 * inf)))}
    return out


def main(path):
    from paper_2106_03452_amd import function as F
    from paper_2106_03452_amd.batch import BatchPlan, Job
    dev = torch.device("cuda", 0)
    t0 = time.time()
    out = {"bars": {"e_chi": 1e-5, "e_dpoints": 1e-4, "e_dnormals": 1e-4,
                    "fd_entry": "|g - g_FD| <= 1e-4 max(|g_FD|, 1e-3 |g|_inf)"},
           "workloads": {}}
    W = out["workloads"]
    say("32^3 sphere, forward")
    W["c1_32_fwd"] = run_pair(F, S.config_c1(), dev, with_target=False)
    say("128^3 torus + sphere, fwd+bwd, finite differences")
    sh = S.config_c2()
    W["c2_128"] = run_pair(F, sh, dev)
    # the adjoint alone: the oracle's G (rounded to FP32) into the GPU backward
    ref, aux = oracle.forward(sh.points, sh.normals, 128, sh.sigma)
    ref_t, _ = oracle.forward(sh.points_clean, sh.normals_clean, 128, sh.sigma)
    G_r = (2.0 * (ref - ref_t) / ref.size).astype(np.float32)
    chi, saved = F.forward(to_dev(sh.points, dev), to_dev(sh.normals, dev), 128, sh.sigma)
    dp, dn = F.backward(chi, saved, to_dev(G_r, dev), sh.P, 128, sh.sigma)
    dc_r, dn_r = oracle.backward(aux, G_r.astype(np.float64))
    W["c2_128"]["adjoint_alone"] = {"e_dpoints": l2_rel(host(dp), dc_r), "e_dnormals": l2_rel(host(dn), dn_r),
                                    "fd": fd_entries(host(dp), host(dn))}
    say("128^3 with half outliers")
    W["c2_128_half_outliers"] = run_pair(F, S.config_c2_outliers(), dev)
    say("256^3 superellipsoid, fwd+bwd")
    W["c3_256"] = run_pair(F, S.config_c3(), dev)
    say("256^3 cloud on 512^3 vs stored oracle samples")
    g = np.load(os.path.join(HERE, "golden", "c3_512_samples.npz"))
    sh = S.config_c3()
    chi, saved = F.forward(to_dev(sh.points, dev), to_dev(sh.normals, dev), 512, sh.sigma)
    G = to_dev(S.loss_gradient(512, 512), dev)
    dp, dn = F.backward(chi, saved, G, sh.P, 512, sh.sigma)
    torch.cuda.synchronize()
    del G
    chi_s = host(chi.reshape(-1)[torch.as_tensor(g["vox"], device=dev)])
    pi = torch.as_tensor(g["pts"], device=dev)
    W["c3_cloud_512_samples"] = {
        "res": 512, "npoints": sh.P, "voxels": int(len(g["vox"])), "points_sampled": int(len(g["pts"])),
        "e_chi": float(np.abs(chi_s - g["chi"]).max() / float(g["chi_max"])),
        "e_dpoints": l2_rel(host(dp[pi]), g["dpoints"]), "e_dnormals": l2_rel(host(dn[pi]), g["dnormals"])}
    del chi, saved, dp, dn
    for res in (64, 128):
        say(f"thin plate {res}^3")
        W[f"thin_plate_{res}"] = run_pair(F, S.thin_plate(7, 60000, res), dev)
    # clouds with random normals: |c| small against max|chi'|, so chi carries
    # chi''s FP32 error amplified by a = max|chi| / m (chi' and c keep 1e-5)
    for res, P in ((16, 600000), (64, 10007)):
        say(f"random normals {res}^3, {P} points")
        sh = S.tiny_case(7 * res + P, res, P, 2.0, kind="uniform")
        chi, saved = F.forward(to_dev(sh.points, dev), to_dev(sh.normals, dev), res, 2.0)
        ref, aux = oracle.forward(sh.points, sh.normals, res, 2.0)
        sc = F.scalars(saved)
        chip = host(chi) / sc["scale"] + sc["mean"]
        W[f"random_normals_{res}_{P}"] = {
            "res": res, "npoints": P, "status": F.status(saved),
            "e_chi_prime": max_rel(chip, aux["chi_prime"]),
            "e_c": abs(sc["cscale"] - aux["cscale"]) / np.abs(aux["chi_prime"]).max(),
            "e_chi_amplified": max_rel(host(chi), ref),
            "amplification": max(1.0, float(np.abs(ref).max() / aux["m"]))}
    say("64-shape batch, per shape")
    shapes = S.config_c4()
    jobs = []
    for s_ in shapes:
        p, n = to_dev(s_.points, dev), to_dev(s_.normals, dev)
        c, _ = F.forward(p, n, s_.res, s_.sigma)
        jobs.append(Job(p, n, s_.res, s_.sigma, (2.0 * c / c.numel()).contiguous()))
    plan = BatchPlan(jobs)
    plan.run()
    torch.cuda.synchronize()
    per = []
    for s_, (chi_b, dp_b, dn_b) in zip(shapes, plan.results()):
        ref, aux = oracle.forward(s_.points, s_.normals, s_.res, s_.sigma)
        dc_r, dn_r = oracle.backward(aux, 2.0 * ref / ref.size)
        per.append({"res": s_.res, "npoints": s_.P, "kind": s_.kind, "e_chi": max_rel(host(chi_b), ref),
                    "e_dpoints": l2_rel(host(dp_b), dc_r), "e_dnormals": l2_rel(host(dn_b), dn_r)})
    W["c4_batch_per_shape"] = {"shapes": per, "max": {k: max(q[k] for q in per)
                                                      for k in ("e_chi", "e_dpoints", "e_dnormals")}}
    # the slab-decomposed forward: the 256^3 workload in 8 slabs against the
    # oracle, the same cloud on 512^3 in 4 slabs against the stored samples,
    # and one Fourier mode on 1024^3 in 8 slabs against its closed form
    from paper_2106_03452_amd import slab as SL
    say("slab forward 256^3 / 8 slabs")
    sh = S.config_c3()
    chi, sc = SL.forward(to_dev(sh.points, dev), to_dev(sh.normals, dev), 256, sh.sigma, 8)
    ref, aux = oracle.forward(sh.points, sh.normals, 256, sh.sigma)
    W["slab_c3_256_8"] = {"res": 256, "npoints": sh.P, "slabs": 8, "status": sc["status"],
                          "e_chi": max_rel(host(chi), ref)}
    say("slab forward 512^3 / 4 slabs vs stored oracle samples")
    chi, sc = SL.forward(to_dev(sh.points, dev), to_dev(sh.normals, dev), 512, sh.sigma, 4)
    chi_s = host(chi.reshape(-1)[torch.as_tensor(g["vox"], device=dev)])
    W["slab_c3_cloud_512_samples"] = {"res": 512, "npoints": sh.P, "slabs": 4, "status": sc["status"],
                                      "e_chi": float(np.abs(chi_s - g["chi"]).max() / float(g["chi_max"]))}
    del chi
    say("slab spectral closed form 1024^3 / 8 slabs")
    res, sigma, k, d = 1024, 2.0, (100, -3, 201), 2
    j = torch.arange(res, device=dev, dtype=torch.float64) * (2 * np.pi / res)
    th = k[0] * j[:, None, None] + k[1] * j[None, :, None] + k[2] * j[None, None, :]
    v = torch.zeros((3, res, res, res), dtype=torch.float32, device=dev)
    v[d] = torch.cos(th).float()
    K2 = float(np.dot(k, k))
    expect = torch.sin(th)
    del th
    expect *= np.exp(-2 * sigma ** 2 * K2 / res ** 2) * k[d] / (2 * np.pi * K2)
    outp = SL.debug_spectral(v, sigma, 8)
    del v
    W["slab_mode_1024_8"] = {"res": res, "slabs": 8, "mode": list(k), "channel": d,
                             "e_chi": float((outp.double() - expect).abs().max() / expect.abs().max())}
    del outp, expect
    torch.cuda.empty_cache()
    out["seconds"] = round(time.time() - t0, 1)
    worst = {}
    for name, w in W.items():
        src = w["max"] if "max" in w else w
        for k in ("e_chi", "e_dpoints", "e_dnormals"):
            if k in src:
                worst[k] = max(worst.get(k, 0.0), src[k])
    out["worst"] = worst
    out["all_within_bars"] = all(worst[k] <= out["bars"][k] for k in worst)
    with open(path, "w") as fh:
        json.dump(out, fh, indent=1)
        fh.write("\n")
    say(f"done in {out['seconds']} s; worst {worst}; within bars: {out['all_within_bars']}")


if __name__ == "__main__":
    main(sys.argv[1] if len(sys.argv) > 1 else "parity_summary.json")
