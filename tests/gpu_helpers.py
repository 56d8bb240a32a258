"""Shared pieces of the GPU parity tests: device upload and the comparison of
one denoised cloud with the oracle.

Bars: sigma_g agrees to FP64 rounding; sigma_est and every filtered colour are
within 1e-3 on the 0..255 scale; q is equal unless the oracle's own losses at
the two values are within the FP32 sweep error (then the output is checked at
the GPU's q).
"""
import math

import numpy as np
import torch

import oracle as O

COLOUR_TOL = 1e-3


def dev(a, dtype):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda")


def oracle_params(prm):
    return dict(bits=prm.bits, num_dirs=prm.num_dirs, window=prm.window, k=prm.k, patch=prm.patch,
                q_max=prm.q_max, fslr_kappa=prm.fslr_kappa, sigma_g=prm.sigma_g, patch_order=prm.patch_order)


def compare_denoise(out, r, xyz, rgb, prm, ores=None, status_mask=~0):
    """out: host float32 [n][3] from the GPU, r: its decoded result."""
    if ores is None:
        ores = O.denoise(xyz, rgb, oracle_params(prm))
    assert abs(r["sigma_est"] - ores["sigma_est"]) <= COLOUR_TOL
    assert math.isclose(r["sigma_g"], ores["sigma_g"], rel_tol=1e-12, abs_tol=1e-300)
    assert r["n_eff"] == ores["n_eff"]
    # FGBD_ST_RELABELED reports how the path ran (an incoherent input order
    # was renumbered along scan order 0), not a property of the result
    from paper_2401_09721_amd import fgbd
    assert (r["status"] & status_mask & ~fgbd.FGBD_ST_RELABELED) == ores["status"]
    q = r["q"]
    if q != ores["q"]:
        en = ores["energies"]
        target = ores["sigma_est"] ** 2
        assert q < len(en), f"GPU q {q} beyond the oracle's stopping point"
        lg, lo = abs(target - en[q]), abs(target - en[ores["q"]])
        assert abs(lg - lo) <= 1e-5 * max(target, 1.0), f"q {q} vs oracle {ores['q']}: not a near-tie"
        ref = O.filter_power(ores["col"], ores["p"], rgb, q)
    else:
        ref = ores["out"]
        assert r["n_fslr"] == ores["n_fslr"]
    err = float(np.max(np.abs(out - ref))) if out.size else 0.0
    assert err <= COLOUR_TOL, f"max colour error {err}"
    return out, r, ores
