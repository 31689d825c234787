"""Shared helpers of the GPU parity tests: build a GPU mesh and an oracle
mesh from the same seeded workload, and compare fields."""
import sys

import numpy as np

import oracle as O


def say(*a):
    """Name the case before a GPU step (flushed, so a crash still shows it)."""
    print("[case]", *a, flush=True)
    sys.stdout.flush()


def oracle_mesh(case, integrator=0):
    return O.Mesh(case.n, case.gamma, case.lo, case.hi, case.bc, integrator=integrator)


def gpu_mesh(case, precision, integrator=0):
    from paper_2501_02317_amd import hydro as H
    h = H.Hydro(case.n, case.gamma, case.cfl, precision=precision, lo=case.lo, hi=case.hi,
                bc=case.bc, integrator=integrator)
    h.set_primitive(case.W)
    return h


def rel_l1(a, ref):
    """Per-component relative L1: sum |a - ref| / sum |ref|."""
    a = a.reshape(a.shape[0], -1)
    ref = ref.reshape(ref.shape[0], -1)
    den = np.abs(ref).sum(axis=1)
    den = np.where(den > 0, den, 1.0)
    return np.abs(a - ref).sum(axis=1) / den


def max_rel(a, ref):
    """Per-component max |a - ref| / max |ref|."""
    a = a.reshape(a.shape[0], -1)
    ref = ref.reshape(ref.shape[0], -1)
    den = np.abs(ref).max(axis=1)
    den = np.where(den > 0, den, 1.0)
    return np.abs(a - ref).max(axis=1) / den


def bitwise_equal(a, b):
    """Every value identical (+0 and -0 count as equal)."""
    return a.shape == b.shape and np.array_equal(a, b)
