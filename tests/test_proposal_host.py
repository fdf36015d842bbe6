"""Host-side logic of the learned proposal (no GPU): the period windows and
their labels, against the oracle's definition of the windows."""

import numpy as np

from oracle import net as onet
from paper_2503_20875_amd.proposal import Windows


def test_windows_match_oracle_definition():
    for n, lo_p, hi_p, bin_days in ((512, 1.0, 100.0, 111.1 / 8192), (48, 0.1, 5.0, 0.02), (7, 0.5, 45.0, 0.3)):
        w = Windows.log_spaced(n, lo_p, hi_p, bin_days)
        q, edges = onet.windows_for(n, lo_p, hi_p)
        assert np.allclose(w.q, q) and np.allclose(w.edges, edges, rtol=1e-15)
        assert np.allclose(w.trials(4), onet.fold_trials(edges, 4, bin_days), rtol=1e-15)


def test_labels_one_window_per_period():
    w = Windows.log_spaced(512, 1.0, 100.0, 0.01)
    periods = np.array([1.0, 3.3, 99.999, 0.5, 150.0])
    y = w.labels(periods)
    assert y.shape == (5, 512)
    assert y[0, 0] == 1 and y[0].sum() == 1  # left edge belongs to window 0
    k = int(np.argmax(y[1]))
    assert w.edges[k] <= 3.3 < w.edges[k + 1]
    assert y[2, 511] == 1
    assert y[3].sum() == 0 and y[4].sum() == 0  # outside the windows


def test_windows_rejects_bad_arguments():
    import pytest
    for args in ((0, 1.0, 2.0, 0.1), (4, 2.0, 1.0, 0.1), (4, 1.0, 2.0, 0.0)):
        with pytest.raises(ValueError):
            Windows.log_spaced(*args)


def test_k_for_recall():
    from paper_2503_20875_amd.learned import k_for_recall
    ranks = [0, 3, 10, 200]
    assert k_for_recall(ranks, 1.0, 512) == 201  # all four inside the top 201
    assert k_for_recall(ranks, 0.75, 512) == 11
    assert k_for_recall(ranks, 0.5, 512) == 4
    assert k_for_recall([], 0.99, 512) == 1
    assert k_for_recall([600], 0.99, 512) == 512  # capped at the number of windows


def test_fallback_threshold():
    from paper_2503_20875_amd.learned import fallback_threshold

    def row(det, rec, snr):
        return dict(detected=det, recalled=rec, restricted_snr=snr)

    rows = [row(True, True, 12.0)] * 97 + [row(True, False, 6.5), row(True, False, 6.9), row(True, False, 5.0),
                                           row(False, False, 9.0)]
    # 100 detections, 3 missed: at 99% one miss may stay, so the two lowest
    # restricted SNRs must fall back; the threshold sits just above 6.5
    tau = fallback_threshold(rows, 0.99)
    assert 6.5 < tau < 6.5 + 1e-12
    assert sum(r["detected"] and (r["recalled"] or r["restricted_snr"] < tau) for r in rows) == 99
    # every miss rescued at a 100% target; none needed at 97%
    assert 6.9 < fallback_threshold(rows, 1.0) < 6.9 + 1e-12
    assert fallback_threshold(rows, 0.97) == float("-inf")
    assert fallback_threshold([row(False, False, 3.0)], 0.99) == float("-inf")
    # a curve where nothing was folded has a restricted SNR of -inf and always falls back
    assert fallback_threshold([row(True, False, float("-inf"))] + [row(True, True, 9.0)] * 3, 1.0) > float("-inf")


def test_store_calibration_keeps_the_arrays(tmp_path):
    """Calibrated operating points go into the archive's metadata; every
    array and the other metadata stay as they were."""
    import json
    from paper_2503_20875_amd.learned import store_calibration
    path = str(tmp_path / "w.npz")
    meta = {"n_event": 8, "hidden": 64, "input": "signed"}
    a = np.arange(12, dtype=np.float32).reshape(3, 4)
    np.savez(path, W0=a, __meta__=np.frombuffer(json.dumps(meta).encode(), dtype=np.uint8))
    store_calibration(path, 89, 6.25, "calibration half of 1000 curves")
    store_calibration(path, 90, None, "again")
    with np.load(path, allow_pickle=False) as z:
        assert np.array_equal(z["W0"], a) and z["W0"].dtype == np.float32
        got = json.loads(bytes(z["__meta__"]).decode())
    assert got == dict(meta, calibrated_k=90, calibrated_fallback_snr=None, calibration="again")


def test_committed_weights_carry_their_operating_points():
    """The default network's archive says which input it was trained on and
    the operating points calibrated for it (read without executing anything
    from the file)."""
    import json
    import os
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    with np.load(os.path.join(root, "paper_2503_20875_amd", "weights", "proposal.npz"), allow_pickle=False) as z:
        meta = json.loads(bytes(z["__meta__"]).decode())
    assert meta["input"] == "signed"
    assert meta["calibrated_k"] == 89
    assert 5.0 < meta["calibrated_fallback_snr"] < 8.0
    with np.load(os.path.join(root, "paper_2503_20875_amd", "weights", "proposal_long.npz"), allow_pickle=False) as z:
        assert json.loads(bytes(z["__meta__"]).decode()).get("input", "abs") in ("abs", "signed")
