"""The C ABI used from a plain host program (tests/c_abi/psr_roundtrip.cpp,
built here with hipcc against include/psr.h and the in-tree libpsr.so): a
forward and a backward through psr_forward / psr_saved_status /
psr_saved_scalars / psr_backward only, checked against the FP64 oracle with
the bars of the Python-path parity tests."""
import os
import shutil
import subprocess

import numpy as np
import pytest

import oracle
import psr_synth as S
from gpu_common import announce, l2_rel, max_rel

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIBDIR = os.path.join(ROOT, "paper_2106_03452_amd")
SRC = os.path.join(ROOT, "tests", "c_abi", "psr_roundtrip.cpp")


@pytest.fixture(scope="module")
def exe(tmp_path_factory):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    assert os.path.exists(os.path.join(LIBDIR, "libpsr.so")), "build libpsr.so first"
    out = str(tmp_path_factory.mktemp("c_abi") / "psr_roundtrip")
    subprocess.run([hipcc, "-O2", "-std=c++17", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
                    "-Wno-unused-command-line-argument", "-I", os.path.join(ROOT, "include"), SRC,
                    "-L", LIBDIR, "-lpsr", f"-Wl,-rpath,{LIBDIR}", "-o", out], check=True, timeout=300)
    return out


def _run(exe, tmp_path, sh, G):
    res, P = sh.res, sh.P
    fin, fout = str(tmp_path / "in.bin"), str(tmp_path / "out.bin")
    with open(fin, "wb") as f:
        f.write(np.int64(P).tobytes() + np.int32(res).tobytes() + np.float32(sh.sigma).tobytes())
        f.write(np.ascontiguousarray(sh.points, np.float32).tobytes())
        f.write(np.ascontiguousarray(sh.normals, np.float32).tobytes())
        f.write(np.ascontiguousarray(G, np.float32).tobytes())
    subprocess.run([exe, fin, fout], check=True, timeout=120)
    raw = open(fout, "rb").read()
    status = int(np.frombuffer(raw[:4], np.int32)[0])
    sc = np.frombuffer(raw[4:36], np.float64)
    o = 36
    chi = np.frombuffer(raw[o:o + 4 * res ** 3], np.float32).reshape(res, res, res)
    o += 4 * res ** 3
    dp = np.frombuffer(raw[o:o + 12 * P], np.float32).reshape(P, 3)
    dn = np.frombuffer(raw[o + 12 * P:o + 24 * P], np.float32).reshape(P, 3)
    return status, sc, chi, dp, dn


@pytest.mark.parametrize("res,P,kind,seed", [(32, 2049, "torus", 3), (64, 4000, "sphere", 5), (256, 20000, "torus", 9)])
def test_c_host_program_matches_oracle(exe, tmp_path, res, P, kind, seed):
    announce(f"C ABI host program res={res} P={P} kind={kind}")
    sh = S.tiny_case(seed, res, P, 2.0, kind=kind)
    G = S.loss_gradient(res, seed + 100)
    status, sc, chi, dp, dn = _run(exe, tmp_path, sh, G)
    ref, aux = oracle.forward(sh.points, sh.normals, res, 2.0)
    dc_r, dn_r = oracle.backward(aux, G.astype(np.float64))
    e_chi, e_dp, e_dn = max_rel(chi, ref), l2_rel(dp, dc_r), l2_rel(dn, dn_r)
    print(f"C ABI res={res}: e_chi={e_chi:.2e} e_dpoints={e_dp:.2e} e_dnormals={e_dn:.2e}")
    assert status == 0
    c = abs(aux["cscale"])
    assert abs(sc[0] - aux["mu"]) <= 1e-5 * c and abs(sc[1] - aux["cscale"]) <= 1e-5 * c
    assert e_chi < 1e-5 and e_dp < 1e-4 and e_dn < 1e-4
