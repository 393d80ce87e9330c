"""Readers of the stored oracle values of the full-size workloads (tests/golden/*.json, written
by tests/golden/make_fullsize_golden.py from oracle/ and the input generator only), and the
FP32-moment error gate that the tests and the benchmark state.

FP32-moment gate (per pair): |dU| <= max(1e-5 |U|, E / 8), E = 2^-24 * sens, where sens is
the oracle's first-order sensitivity of eq. (9) to moment errors at the scale of the
absolute sums (sum over the terms of |factor| (Abar^A |Q^B| + |Q^A| Abar^B)).  1e-5 |U| is the
relative gate fixed before any measurement; E is the a-priori size of the error of a moment
pass that is off by one FP32 rounding of each moment's absolute sum, and bounds what any
FP32 moment pass can promise when |U| is far below the magnitude of its terms (neutral
molecules whose terms cancel).  Measured on MI355X: at most 0.036 E over the 1024 pairs of
the uneven batch for every FP32 run length from 8 to 256 atoms per thread, 0.0042 E over the
4096 poses of the orientation scan."""
import json
import os

import numpy as np

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
U32 = 2.0 ** -24
REL_GATE = 1e-5
E_FRACTION = 1.0 / 8.0


def load(name):
    with open(os.path.join(GOLDEN, name + ".json")) as f:
        return json.load(f)


def same_fragment(rec, x, q):
    """The stored fragment record matches these atoms (count, sums of coordinates and charges)."""
    return (rec["n"] == len(q) and np.isclose(rec["sum_xyz"], float(np.sum(x)), rtol=1e-12, atol=0)
            and np.isclose(rec["sum_q"], float(np.sum(q)), rtol=1e-12, atol=1e-12 * rec["sum_abs_q"]))


def fp32_gate(U, sens):
    return np.maximum(REL_GATE * np.abs(U), E_FRACTION * U32 * np.asarray(sens))


def error_statement(U_gpu, U_ref, abs_sum, sens):
    """The FP32 error statement of a set of pairs: max and p99 of |dU|/|U|, max of
    |dU|/abs_sum, the a-priori estimate E = 2^-24 sens relative to |U| (median, max), the
    measured error as a fraction of E, and the pairs that miss the relative gate."""
    U_gpu, U_ref = np.asarray(U_gpu), np.asarray(U_ref)
    abs_sum, sens = np.asarray(abs_sum), np.asarray(sens)
    d = np.abs(U_gpu - U_ref)
    rel = d / np.abs(U_ref)
    E = U32 * sens
    miss = np.nonzero(rel > REL_GATE)[0]
    return {"pairs": int(len(d)), "max_rel": float(rel.max()), "p99_rel": float(np.percentile(rel, 99)),
            "median_rel": float(np.median(rel)), "max_err_over_abs_terms": float(np.max(d / abs_sum)),
            "apriori_E_over_U": {"median": float(np.median(E / np.abs(U_ref))), "max": float(np.max(E / np.abs(U_ref)))},
            "err_over_E": {"median": float(np.median(d / E)), "max": float(np.max(d / E))},
            "within_gate": int(np.sum(d <= fp32_gate(U_ref, sens))),
            "missing_rel_gate": [{"index": int(i), "rel": float(rel[i]), "U_over_abs_terms": float(abs(U_ref[i]) / abs_sum[i]),
                                  "E_over_U": float(E[i] / abs(U_ref[i]))} for i in miss]}
