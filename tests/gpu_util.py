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
