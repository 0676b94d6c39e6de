"""Field-by-field comparison of a GPU profile with the oracle's (shared by
the GPU test modules and smoke()).

Everything the method computes is integer, so every comparison is exact:
sample records, tracked objects, the twelve per-line arrays, scalars, leak
rationals and gates.
"""
import numpy as np

import oracle

KEYS = ("final_F", "peak_F", "peak_sampled_F", "threshold_used", "K", "H")
LINE_ARRAYS = oracle.HIST_NAMES + ("lap_num", "lap_den", "lit_num", "lit_den", "lap_gate", "lit_gate")


def compare(g, o, label=""):
    assert g["status"] == o["status"], (label, g["status"], o["status"])
    if o["status"] != oracle.OK:
        return
    for k in KEYS:
        assert g[k] == o[k], (label, k, g[k], o[k])
    gs, os_ = g["samples"], o["samples"]
    assert gs.shape == os_.shape, (label, gs.shape, os_.shape)
    for f in ("event_idx", "line", "F", "py", "nat"):
        if not np.array_equal(gs[f], os_[f]):
            bad = np.flatnonzero(gs[f] != os_[f])[:5]
            raise AssertionError(f"{label}: samples.{f} differ at {bad}: gpu {gs[bad]} oracle {os_[bad]}")
    for f in ("event_idx", "line", "ptr", "freed"):
        assert np.array_equal(g["tracked"][f], o["tracked"][f]), (label, "tracked", f)
    for name in LINE_ARRAYS:
        if not np.array_equal(g[name], o[name]):
            bad = np.flatnonzero(g[name] != o[name])[:5]
            raise AssertionError(f"{label}: {name} differs at lines {bad}: gpu {g[name][bad]} oracle {o[name][bad]}")
