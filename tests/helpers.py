"""Shared helpers of the GPU parity tests: inputs, layout conversion, error norms.

The oracle and the HIP library share nothing but the seeded inputs; the
conversions between their layouts live here and in the binding, not in either.
"""
import numpy as np

from paper_1612_06424_amd.inputs import gaussian_field, random_links  # noqa: F401


def relerr(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


def lib():
    import paper_1612_06424_amd.dd as dd
    return dd


def step(msg):
    """Name the case before a GPU step (flushed, so a crash still shows it)."""
    print(f"[gpu-step] {msg}", flush=True)
