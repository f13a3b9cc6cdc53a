"""Shared helpers of the GPU parity tests (inputs from ntf_synth, expected
values from the oracle only)."""
import numpy as np

import ntf_synth
from oracle import ntf_oracle as orc


def rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


def problem(dims, F, seed, f64, snr_db=20.0, dist="uniform", clip=False):
    dt = np.float64 if f64 else np.float32
    pt = ntf_synth.planted(dims, F, seed, snr_db=snr_db, dist=dist, clip=clip, dtype=dt)
    H0 = ntf_synth.init_factors(dims, F, seed, dtype=dt)
    return pt, H0


def to_dev(arrs, dev):
    import torch
    return [torch.from_numpy(np.ascontiguousarray(a)).to(dev) for a in arrs]


def oracle_steps(X, H0, steps, opts, paper=False, rho=None):
    st = orc.init_state([np.asarray(h, dtype=np.float64) for h in H0], rho0=opts.rho0, paper=paper)
    if rho is not None:
        st.rho = list(rho)
    for _ in range(steps):
        orc.outer_step(np.asarray(X, dtype=np.float64), st, opts)
    return st
