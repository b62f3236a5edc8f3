"""Shared helpers of the GPU parity tests (no method arithmetic here)."""
import numpy as np

from oracle import fields as F

KEYS = ("Ms", "A", "D", "Ku", "u", "H", "alpha")


def oracle_params(p, terms, gamma=2.21e5):
    return F.Params(terms=terms, gamma=gamma, **{k: p[k] for k in KEYS if k in p})


def gpu_params(mm, p, terms, gamma=2.21e5):
    return mm.make_params(terms=terms, gamma=gamma, **{k: p[k] for k in KEYS if k in p})


def field_err(got, ref):
    """max_i |got_i - ref_i| / max_i |ref_i| over cells (vectors along axis 0)."""
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    d = np.sqrt(np.sum((got - ref) ** 2, axis=0))
    r = np.sqrt(np.sum(ref ** 2, axis=0))
    return float(np.max(d) / np.max(r))


def to_dev(a, dtype):
    import torch
    return torch.tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda")


def representable(m, dtype):
    """m rounded to the device precision, returned as float64 (the oracle's input)."""
    import torch
    return torch.tensor(m, dtype=dtype).double().numpy()
