"""Shared helpers for the tests (not a test module)."""
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def load_package():
    """Import the binding, building libgrav.so first only if it is absent."""
    lib = os.path.join(ROOT, "paper_2602_03857_amd", "libgrav.so")
    if not os.path.exists(lib):
        # by path: importing the package would try to load the missing library
        import importlib.util
        spec = importlib.util.spec_from_file_location(
            "grav_build", os.path.join(ROOT, "paper_2602_03857_amd", "build.py"))
        mod = importlib.util.module_from_spec(spec)
        spec.loader.exec_module(mod)
        mod.build()
    import paper_2602_03857_amd as g
    return g


def rel_l2(got, ref) -> float:
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    return float(np.linalg.norm(got - ref) / np.linalg.norm(ref))


def to_np(t):
    return t.detach().cpu().numpy()
