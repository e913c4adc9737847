"""FP64 CPU oracle for snippet-based labelling and its per-element F1 score.

TEST INFRASTRUCTURE ONLY, like the rest of ``oracle``: the product path never
imports it and it shares no code with the GPU library.

The paper scores a labelling of the series element by element against the
true labelling with precision TP/(TP+FP), recall TP/(TP+FN) and their harmonic
mean F1 (section 5.2, the accuracy experiment).  It does not spell out how the
snippets turn into element labels; the reading used here (also listed in the
design notes) is:

  * element t takes the snippet that owns window t (eq. 6: the window's
    nearest snippet); the elements after the last window start, t > n-m,
    take the owner of the last window;
  * each snippet stands for the true class held by most of the elements it
    labels (ties to the lowest class);
  * precision, recall and F1 are per true class, with 0 where a denominator is
    0; the summary is their mean over the classes present in the truth.
"""
from __future__ import annotations

import numpy as np


def element_labels(owner: np.ndarray, n: int, m: int) -> np.ndarray:
    """Snippet (greedy rank) labelling each element t < n."""
    owner = np.asarray(owner)
    Nm = n - m + 1
    assert owner.shape == (Nm,)
    lab = np.empty(n, dtype=np.int64)
    for t in range(n):
        lab[t] = owner[min(t, Nm - 1)]
    return lab


def confusion(pred: np.ndarray, truth: np.ndarray, K: int, C: int) -> np.ndarray:
    """conf[p, c] = number of elements labelled by snippet p whose true class is c."""
    conf = np.zeros((K, C), dtype=np.int64)
    for p, c in zip(pred, truth):
        conf[int(p), int(c)] += 1
    return conf


def majority_map(conf: np.ndarray) -> np.ndarray:
    """Class each snippet stands for: the most frequent true class among its
    elements, ties to the lowest class (a snippet with no elements maps to 0)."""
    K, C = conf.shape
    out = np.zeros(K, dtype=np.int64)
    for p in range(K):
        best = 0
        for c in range(1, C):
            if conf[p, c] > conf[p, best]:
                best = c
        out[p] = best
    return out


def f1_scores(truth: np.ndarray, predicted_class: np.ndarray, C: int):
    """Per-class precision, recall, F1 of a labelling, and the mean F1 over the
    classes that occur in the truth."""
    prec = np.zeros(C)
    rec = np.zeros(C)
    f1 = np.zeros(C)
    present = []
    for c in range(C):
        tp = int(np.sum((predicted_class == c) & (truth == c)))
        fp = int(np.sum((predicted_class == c) & (truth != c)))
        fn = int(np.sum((predicted_class != c) & (truth == c)))
        prec[c] = tp / (tp + fp) if tp + fp > 0 else 0.0
        rec[c] = tp / (tp + fn) if tp + fn > 0 else 0.0
        f1[c] = 2 * prec[c] * rec[c] / (prec[c] + rec[c]) if prec[c] + rec[c] > 0 else 0.0
        if tp + fn > 0:
            present.append(c)
    macro = float(np.mean(f1[present])) if present else 0.0
    return prec, rec, f1, macro


def label_f1(owner: np.ndarray, truth: np.ndarray, m: int, K: int, C: int):
    """The whole labelling score: element labels, majority map, F1."""
    truth = np.asarray(truth)
    n = len(truth)
    pred = element_labels(owner, n, m)
    conf = confusion(pred, truth, K, C)
    mp = majority_map(conf)
    prec, rec, f1, macro = f1_scores(truth, mp[pred], C)
    return dict(conf=conf, map=mp, precision=prec, recall=rec, f1=f1, macro_f1=macro)
