"""Inputs as a context stores them.

A context of FP32 precision keeps positions and velocities in float32
(round to nearest even on the host when the state is set).  Tests hand the
oracle the same rounded values, computed here on the host, so that no oracle
input is read back from the device; the tests also check that the device
state equals them exactly.
"""
import numpy as np


def as_stored(a, fp32: bool) -> np.ndarray:
    a = np.ascontiguousarray(a, np.float64)
    return np.ascontiguousarray(a.astype(np.float32).astype(np.float64)) if fp32 else a
