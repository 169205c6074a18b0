"""The oracle's per-part results and the checks of GPU results against them.

Shared by the full-size parity test, the record generator under
tests/golden/full_size/ and the served-results test.  The records are the
oracle's own (its samples, its bits, its statistics, class and setups); the
checks allow exactly what grazing rays and flagged ties leave open:
  - accessibility by the grazing rays over S N (and never more than 1e-4);
  - a dominant-axis share by (T + 2G) over the included samples, T the
    oracle's flagged ties, G the rows holding a grazing ray (such a row's
    free count and axis may differ, and it may move in or out of the
    included samples);
  - the mean concentration by 1e-4 (FP32 sums) plus the same fraction;
  - the class exactly when no allowance reaches a threshold;
  - the histogram by 2e-4 of its mass (bin edges) plus the grazing rays;
  - setups exactly when no six-axis ray is grazing, else code counts within
    two per affected row and the minimum exact on the GPU's own codes.
"""
from __future__ import annotations

import numpy as np

THRESHOLDS = {"access": 0.60, "share": 0.45, "conc": 0.40}


def stats_record(orc, samples, dirs, bits, grazing_rows, hist=True):
    """Section 3.3 indicators and class from the oracle's bits."""
    N = len(dirs)
    st = orc.dirstats(samples, dirs, bits)
    cnt = orc.counts(bits, N)
    ind = orc.indicators(cnt, N, st["axis"], st["conc"])
    multi, tripped = orc.classify(ind)
    rec = {"access": ind["access"], "shares": ind["shares"], "conc": ind["conc"],
           "n_included": ind["n_included"], "n_blind": ind["n_blind"],
           "n_ties": int(st["tie"].sum()), "rows_with_grazing": int(len(np.unique(np.asarray(grazing_rows)))),
           "multi_axis": bool(multi), "tripped": int(tripped)}
    return rec, (st["hist"].astype(np.int64) if hist else None)


def setups_record(orc, mesh, samples, axes_bits, tool):
    """Section 3.3 (last paragraph): reach, classes and setups from the
    oracle's six-axis bits."""
    bbox, diag, _ = orc.mesh_info(mesh.verts)
    cls, code = orc.reach_classes(samples["point"], samples["tri"], np.asarray(axes_bits)[:, 0], bbox,
                                  orc.bbox_face_tris(mesh.verts, mesh.tris, bbox, diag), tool)
    h = orc.code_histogram(cls, code)
    mn = orc.min_setups_exact(h)
    gr = orc.min_setups_greedy(h) if h.sum() else (0, 0)
    return {"tool_length": tool, "min_count": mn[0], "min_mask": mn[1], "greedy_count": gr[0],
            "greedy_mask": gr[1], "n_class": [int((cls == k).sum()) for k in range(4)],
            "code_hist": [int(x) for x in h]}


def check_class(rep, o, n_grazing, S, N):
    """GPU class report `rep` (hra.Context.classify) against the oracle's
    stats record `o`, whose bits had n_grazing grazing rays."""
    G, T = o["rows_with_grazing"], o["n_ties"]
    n_inc = max(1, o["n_included"] - G)
    assert abs(rep["access"] - o["access"]) <= n_grazing / (S * N) + 1e-12
    assert abs(rep["access"] - o["access"]) <= 1e-4
    tol_share = (T + 2 * G) / n_inc
    for k in range(3):
        assert abs(rep["shares"][k] - o["shares"][k]) <= tol_share + 1e-12, (k, rep["shares"], o["shares"], T, G)
    assert abs(rep["conc"] - o["conc"]) <= 1e-4 + (T + 2 * G) / n_inc
    assert abs(rep["n_blind"] - o["n_blind"]) <= G
    if rep["near_tie"]:
        return
    margin = min(abs(o["access"] - THRESHOLDS["access"]), abs(max(o["shares"]) - THRESHOLDS["share"]),
                 abs(o["conc"] - THRESHOLDS["conc"]))
    if T + 2 * G == 0 or margin > 1e-4 + tol_share:
        assert rep["multi_axis"] == o["multi_axis"]


def check_hist(hist, oh, n_free, n_grazing):
    gh = np.asarray(hist).astype(np.int64)
    assert gh.sum() == n_free
    assert np.abs(gh - oh).sum() <= 2e-4 * oh.sum() + n_grazing


def check_setups(orc, su, o, axes_grazing_rows):
    """GPU setup report `su` against the oracle's setups record `o`."""
    got = {k: su[k] for k in ("min_count", "min_mask", "greedy_count", "greedy_mask")}
    got["n_class"], got["code_hist"] = list(su["n_class"]), list(su["code_hist"])
    if len(axes_grazing_rows) == 0:
        for k in ("min_count", "min_mask", "greedy_count", "greedy_mask", "n_class", "code_hist"):
            assert got[k] == o[k], (k, got[k], o[k])
    else:
        g = len(set(int(r) for r in axes_grazing_rows))
        assert np.abs(np.array(got["code_hist"]) - np.array(o["code_hist"])).sum() <= 2 * g
        assert np.abs(np.array(got["n_class"]) - np.array(o["n_class"])).sum() <= 2 * g
        assert (got["min_count"], got["min_mask"]) == orc.min_setups_exact(np.array(got["code_hist"]))
