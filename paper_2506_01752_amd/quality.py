"""Agreement between a found partition and a reference partition (section 5's evaluation
measures): normalised mutual information, adjusted mutual information, adjusted Rand index
and pair-counting F1, plus the modularity of a front point. Host-side numpy; these are
reporting tools, not the search.

Partitions are integer label arrays of equal length; label values are arbitrary names.
"""
from __future__ import annotations

import numpy as np


def _contingency(a, b):
    a = np.asarray(a).ravel()
    b = np.asarray(b).ravel()
    if a.shape != b.shape:
        raise ValueError("partitions of different sizes")
    _, ia = np.unique(a, return_inverse=True)
    _, ib = np.unique(b, return_inverse=True)
    ka, kb = ia.max() + 1, ib.max() + 1
    cell = np.bincount(ia.astype(np.int64) * kb + ib, minlength=ka * kb).reshape(ka, kb)
    return cell.astype(np.float64)


def _entropy(counts, n):
    p = counts[counts > 0] / n
    return float(-(p * np.log(p)).sum())


def nmi(a, b) -> float:
    """Mutual information over the arithmetic mean of the two entropies (1 for equal
    partitions up to renaming; 1 also when both are a single community)."""
    c = _contingency(a, b)
    n = c.sum()
    ha, hb = _entropy(c.sum(1), n), _entropy(c.sum(0), n)
    if ha == 0.0 and hb == 0.0:
        return 1.0
    nz = c > 0
    pij = c[nz] / n
    pa = (c.sum(1, keepdims=True) / n * np.ones_like(c))[nz]
    pb = (c.sum(0, keepdims=True) / n * np.ones_like(c))[nz]
    mi = float((pij * np.log(pij / (pa * pb))).sum())
    return max(0.0, mi / (0.5 * (ha + hb)))


def _expected_mi(ra, rb, n):
    """E[MI] between two partitions with row sizes ra and column sizes rb when one of them is
    relabelled by a uniformly random permutation of the n items: each cell count follows a
    hypergeometric law (Vinh, Epps and Bailey 2010). Sizes that repeat are summed once, with
    their multiplicity."""
    from scipy.special import gammaln
    ua, ma = np.unique(ra.astype(np.int64), return_counts=True)
    ub, mb = np.unique(rb.astype(np.int64), return_counts=True)
    emi = 0.0
    y = ub.astype(np.float64)[:, None]
    for x, mx in zip(ua.astype(np.float64), ma):
        top = min(x, float(ub.max()))
        k = np.arange(1.0, top + 1.0)[None, :]
        ok = (k >= np.maximum(1.0, x + y - n)) & (k <= np.minimum(x, y))
        kk = np.where(ok, k, 1.0)
        logp = (gammaln(x + 1) + gammaln(y + 1) + gammaln(n - x + 1) + gammaln(n - y + 1)
                - gammaln(n + 1) - gammaln(kk + 1) - gammaln(x - kk + 1)
                - gammaln(np.where(ok, y - kk, 0.0) + 1)
                - gammaln(np.where(ok, n - x - y + kk, 0.0) + 1))
        logp = np.where(ok, logp, -np.inf)
        term = np.where(ok, kk / n * np.log(n * kk / (x * y)) * np.exp(logp), 0.0)
        emi += float(mx) * float((mb[:, None] * term).sum())
    return emi


def ami(a, b) -> float:
    """Adjusted mutual information with the max normalisation of section 5:
    (MI - E[MI]) / (max(H(a), H(b)) - E[MI]); 1 for equal partitions up to renaming, 0 on
    average for independent ones."""
    c = _contingency(a, b)
    n = c.sum()
    ra, rb = c.sum(1), c.sum(0)
    if (len(ra) == 1 and len(rb) == 1) or (len(ra) == n and len(rb) == n):
        return 1.0
    ha, hb = _entropy(ra, n), _entropy(rb, n)
    nz = c > 0
    pij = c[nz] / n
    pa = (ra[:, None] / n * np.ones_like(c))[nz]
    pb = (rb[None, :] / n * np.ones_like(c))[nz]
    mi = float((pij * np.log(pij / (pa * pb))).sum())
    emi = _expected_mi(ra, rb, n)
    den = max(ha, hb) - emi
    if den == 0.0:
        return 1.0
    return float((mi - emi) / den)


def _pairs(x):
    return x * (x - 1) / 2.0


def ari(a, b) -> float:
    """Adjusted Rand index (Hubert and Arabie)."""
    c = _contingency(a, b)
    n = c.sum()
    s_ij = _pairs(c).sum()
    s_a, s_b = _pairs(c.sum(1)).sum(), _pairs(c.sum(0)).sum()
    expected = s_a * s_b / _pairs(n) if n > 1 else 0.0
    top = 0.5 * (s_a + s_b)
    if top == expected:
        return 1.0
    return float((s_ij - expected) / (top - expected))


def pair_f1(found, truth) -> float:
    """F1 over node pairs: a pair is positive when both nodes share a community."""
    c = _contingency(found, truth)
    tp = _pairs(c).sum()
    pos_found = _pairs(c.sum(1)).sum()
    pos_truth = _pairs(c.sum(0)).sum()
    if pos_found == 0 and pos_truth == 0:
        return 1.0
    return float(2 * tp / (pos_found + pos_truth))


def modularity(f1: float, f2: float) -> float:
    """Q = (1 - f1) - f2 (Alg. 3's selection criterion, eq. modularity)."""
    return (1.0 - f1) - f2
