"""Pins of the labelling / F1 oracle (CPU only).

The F1 of the oracle is checked against scikit-learn's independent
implementation of the same per-class definition, on random labellings; the
element labelling and the majority map against hand-worked cases."""
import numpy as np
import pytest

from oracle import labelling as LB


def test_element_labels_tail_takes_last_window():
    owner = np.array([0, 0, 1, 2])              # n - m + 1 = 4 windows
    lab = LB.element_labels(owner, n=7, m=4)    # elements 4..6 follow window 3
    assert lab.tolist() == [0, 0, 1, 2, 2, 2, 2]


def test_majority_map_ties_to_lowest_class():
    conf = np.array([[3, 5, 5], [0, 0, 0], [2, 1, 0]])
    assert LB.majority_map(conf).tolist() == [1, 0, 0]


def test_perfect_and_swapped_labelling():
    truth = np.repeat(np.arange(3), 10)
    owner_ok = truth.copy()                      # m = 1: one window per element
    r = LB.label_f1(owner_ok, truth, m=1, K=3, C=3)
    assert r["macro_f1"] == 1.0 and r["map"].tolist() == [0, 1, 2]
    # snippets numbered differently from the classes: the majority map undoes it
    r = LB.label_f1((truth + 1) % 3, truth, m=1, K=3, C=3)
    assert r["macro_f1"] == 1.0 and r["map"].tolist() == [2, 0, 1]


def test_hand_worked_scores():
    # truth: 4 of class 0, 4 of class 1; one snippet labels everything
    truth = np.array([0, 0, 0, 0, 1, 1, 1, 1])
    r = LB.label_f1(np.zeros(8, dtype=int), truth, m=1, K=1, C=2)
    # map -> class 0 (tie 4:4 to the lowest); class 0: P = 4/8, R = 1; class 1: 0
    assert r["map"].tolist() == [0]
    assert r["precision"][0] == 0.5 and r["recall"][0] == 1.0
    assert abs(r["f1"][0] - 2 / 3) < 1e-15 and r["f1"][1] == 0.0
    assert abs(r["macro_f1"] - 1 / 3) < 1e-15


@pytest.mark.parametrize("seed", [0, 1, 2, 3])
def test_f1_matches_sklearn(seed):
    from sklearn.metrics import f1_score, precision_score, recall_score
    rng = np.random.default_rng(seed)
    C, n = 5, 400
    truth = rng.integers(0, C, n)
    truth[truth == 4] = 3                        # class 4 absent from the truth
    pred = np.where(rng.random(n) < 0.6, truth, rng.integers(0, C, n))
    prec, rec, f1, macro = LB.f1_scores(truth, pred, C)
    labels = list(range(C))
    np.testing.assert_allclose(prec, precision_score(truth, pred, labels=labels, average=None, zero_division=0))
    np.testing.assert_allclose(rec, recall_score(truth, pred, labels=labels, average=None, zero_division=0))
    np.testing.assert_allclose(f1, f1_score(truth, pred, labels=labels, average=None, zero_division=0))
    present = sorted(set(truth.tolist()))
    assert abs(macro - f1_score(truth, pred, labels=present, average="macro", zero_division=0)) < 1e-12


def test_planted_mistake_is_caught():
    # counting a false positive as a true positive must change the score
    rng = np.random.default_rng(7)
    truth = rng.integers(0, 3, 200)
    pred = np.where(rng.random(200) < 0.7, truth, rng.integers(0, 3, 200))
    from sklearn.metrics import f1_score
    ref = f1_score(truth, pred, labels=[0, 1, 2], average=None, zero_division=0)
    wrong = np.zeros(3)
    for c in range(3):
        tp = np.sum(pred == c)                  # mistake: every prediction a hit
        fn = np.sum((pred != c) & (truth == c))
        p, r = 1.0, tp / (tp + fn)
        wrong[c] = 2 * p * r / (p + r)
    assert not np.allclose(wrong, ref)
    _, _, f1, _ = LB.f1_scores(truth, pred, 3)
    np.testing.assert_allclose(f1, ref)
