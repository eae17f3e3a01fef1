"""Detection error rates on the host (measurement helpers, not on the hot path).

P_MD = #{active, not detected} / #{active}; P_FA = #{inactive, detected} /
#{inactive}; detection is score >= theta (the threshold module of the
paper's Sec. III-A).  The operating point is the equal-error threshold.
"""
from __future__ import annotations

import numpy as np


def equal_error_point(scores, truth):
    """Threshold among the distinct scores where P_MD and P_FA are closest;
    ties broken by the smaller mean (P_MD + P_FA)/2, then the larger
    threshold.  Returns (eer, theta, p_md, p_fa), eer = (P_MD + P_FA)/2."""
    s = np.asarray(scores, dtype=np.float64).ravel()
    t = np.asarray(truth).ravel().astype(bool)
    n_act = max(int(t.sum()), 1)
    n_ina = max(int((~t).sum()), 1)
    cand = np.unique(s)                                   # ascending
    # count of actives / inactives with score < theta, for each candidate
    act_sorted = np.sort(s[t])
    ina_sorted = np.sort(s[~t])
    miss = np.searchsorted(act_sorted, cand, side="left")                  # active & s < theta
    fa = len(ina_sorted) - np.searchsorted(ina_sorted, cand, side="left")  # inactive & s >= theta
    pmd = miss / n_act
    pfa = fa / n_ina
    gap = np.abs(pmd - pfa)
    mean = 0.5 * (pmd + pfa)
    order = np.lexsort((-cand, mean, gap))                # primary key last
    k = int(order[0])
    return float(mean[k]), float(cand[k]), float(pmd[k]), float(pfa[k])


def error_rate(scores, truth, theta):
    """||alpha_hat - alpha||_1 / (N I) at threshold theta."""
    det = np.asarray(scores) >= theta
    return float(np.mean(det != np.asarray(truth).astype(bool)))
