"""Shared helpers for the GPU parity tests: error metrics against the oracle."""
import numpy as np

# Tolerances of the parity contract: max |df| / rms|f| and per-atom relative
# energy, FP64 mode and mixed mode.
TOL = {
    "fp64": {"force": 1e-10, "energy": 1e-12},
    "mixed": {"force": 1e-5, "energy": 1e-7},
}


def force_error(f, f_ref):
    """max_i |f_i - f_ref_i|_2 / sqrt(mean_i |f_ref_i|^2)."""
    rms = np.sqrt(np.mean(np.sum(f_ref**2, 1)))
    return np.max(np.linalg.norm(f - f_ref, axis=1)) / rms


def energy_error(e, e_ref):
    return np.max(np.abs(e - e_ref) / np.abs(e_ref))


def announce(msg):
    print(f"[gpu-test] {msg}", flush=True)
