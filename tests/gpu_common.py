"""Helpers shared by the GPU parity tests (no solver arithmetic here)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")


def require_gpu():
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return torch.device("cuda", 0)


def to_dev(a, dev):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(dev)


def host(t):
    return t.detach().cpu().numpy().astype(np.float64)


def max_rel(gpu, ref):
    """max |gpu - ref| / max |ref|  (the e_chi metric)."""
    ref = np.asarray(ref, dtype=np.float64)
    return float(np.abs(np.asarray(gpu, dtype=np.float64) - ref).max() / max(np.abs(ref).max(), 1e-300))


def l2_rel(gpu, ref):
    """||gpu - ref||_2 / ||ref||_2  (the e_g metric)."""
    ref = np.asarray(ref, dtype=np.float64)
    return float(np.linalg.norm(np.asarray(gpu, dtype=np.float64) - ref) / max(np.linalg.norm(ref), 1e-300))


def announce(msg):
    print(f"[gpu-case] {msg}", flush=True)
