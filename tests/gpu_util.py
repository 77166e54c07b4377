"""Shared helpers of the GPU tests (inputs and comparisons only)."""
import json
import os

import numpy as np

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def rel(a, b):
    a = np.asarray(a, dtype=np.complex128)
    b = np.asarray(b, dtype=np.complex128)
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / (nb if nb > 0 else 1.0))


def golden_workload(name):
    with open(os.path.join(GOLDEN, "workloads.json")) as f:
        return json.load(f)["workloads"][name]


def device(x):
    import torch
    x = np.ascontiguousarray(x)
    if x.dtype == np.uint16:           # moved as raw 16-bit words; the library reads the bytes
        x = x.view(np.int16)
    t = torch.from_numpy(x).to("cuda")
    torch.cuda.synchronize()
    return t


def say(msg):
    print(msg, flush=True)


# The zero frequency carries almost all of the energy of D, A and the displayed image
# (D[0] over 99% of ||D||^2 on these workloads), so a relative error of the whole array
# bounds the reconstructed signal only loosely.  These compare the whole array and the
# part without the zero frequency, and return the larger error.

def rel_d(got, ref):
    """D on the kept frequencies (index 0 is v = 0)."""
    got, ref = np.asarray(got), np.asarray(ref)
    return max(rel(got, ref), rel(got[1:], ref[1:]))


def rel_a(got, ref):
    """A [n_freq, K] (row 0 is v = 0)."""
    got, ref = np.asarray(got), np.asarray(ref)
    return max(rel(got, ref), rel(got[1:], ref[1:]))


def rel_img(got, ref):
    """The displayed object, whole and minus its mean (the mean is D[0] / sqrt(S |D[0]|))."""
    got = np.asarray(got, dtype=np.complex128)
    ref = np.asarray(ref, dtype=np.complex128)
    return max(rel(got, ref), rel(got - got.mean(), ref - ref.mean()))
