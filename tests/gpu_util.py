"""Helpers shared by the GPU tests (no method arithmetic here)."""
import numpy as np
import pytest
import torch

import oracle


def need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def dev_soa(soa_np):
    return torch.from_numpy(np.ascontiguousarray(soa_np, dtype=np.float32)).cuda()


def dev_globals(g):
    return torch.tensor(np.asarray(g, dtype=np.float32), device="cuda")


def oracle_optics(spec):
    return oracle.Optics(mode=spec.mode, wavelength_um=spec.wavelength_um, na=spec.na,
                         n_medium=spec.n_medium, pixel_um=spec.pixel_um,
                         shear_angle_rad=spec.shear_angle_rad, tilt_fx=spec.tilt_fx,
                         tilt_fy=spec.tilt_fy, photons_mean=spec.photons_mean, seed=spec.seed)


def rel_l2(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def say(*a):
    print(*a, flush=True)
