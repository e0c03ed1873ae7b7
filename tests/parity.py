"""Comparison helpers: GPU result vs the CPU oracle, element by element.

Integers (source, target, delay, group offsets) must match bit for bit.
Weights are fp32 on the GPU and fp64 in the oracle; the bound is
    |w_gpu - w_ref| <= 1e-6 * (|base| + |w_ref - base|)
with base = the mean (normal) or the lower bound (uniform) or the constant:
the GPU evaluates log, sqrt and cospi in fp32 (a few ulp each, about 4e-7
relative on sd*z) and rounds the result to fp32 (6e-8 relative), so the
bound holds with margin; it is relative to the size of both terms of the
weight, so it stays meaningful when the mean is zero.
"""
from __future__ import annotations

import numpy as np

WEIGHT_RTOL = 1e-6


def weight_base(call) -> float:
    kind = call.weight[0]
    return float(call.weight[1])


def per_record_base(calls, creation_index=None) -> np.ndarray:
    counts = np.array([c.n_syn() for c in calls], dtype=np.int64)
    bases = np.repeat(np.array([weight_base(c) for c in calls]), counts)
    return bases if creation_index is None else bases[creation_index.astype(np.int64)]


def check_weights(w_gpu, w_ref, base, where=""):
    w_gpu = np.asarray(w_gpu, dtype=np.float64)
    err = np.abs(w_gpu - w_ref)
    tol = WEIGHT_RTOL * (np.abs(base) + np.abs(w_ref - base))
    bad = np.nonzero(err > tol)[0]
    assert bad.size == 0, (f"{where}: {bad.size} weights outside tolerance; first at {bad[0]}: "
                           f"gpu={w_gpu[bad[0]]!r} ref={w_ref[bad[0]]!r} tol={tol[bad[0]]!r}")


def check_equal(a, b, name):
    a = np.asarray(a).astype(np.int64)
    b = np.asarray(b).astype(np.int64)
    assert a.shape == b.shape, f"{name}: shape {a.shape} vs {b.shape}"
    bad = np.nonzero(a != b)[0]
    assert bad.size == 0, f"{name}: {bad.size} mismatches, first at {bad[0]}: gpu={a[bad[0]]} ref={b[bad[0]]}"


def check_creation_order(gpu, ref, calls):
    check_equal(gpu["src"], ref["src"], "src")
    check_equal(gpu["tgt"], ref["tgt"], "tgt")
    check_equal(gpu["delay"], ref["delay"], "delay")
    check_weights(gpu["w"], ref["w"], per_record_base(calls), "w")


def check_calibrated(gpu, gp, gs, ref, calls):
    check_equal(gpu["src"], ref["s_src"], "sorted src")
    check_equal(gpu["tgt"], ref["s_tgt"], "sorted tgt")
    check_equal(gpu["delay"], ref["s_delay"], "sorted delay")
    check_weights(gpu["w"], ref["s_w"], per_record_base(calls, ref["perm"]), "sorted w")
    check_equal(gp, ref["group_ptr"], "group_ptr")
    check_equal(gs, ref["group_start"], "group_start")
