"""Normalised mutual information between two labelings (test-only).

The accuracy measure of Sec. 5; arithmetic-mean normalisation
NMI = I(a; b) / ((H(a) + H(b)) / 2), computed from the contingency table.
"""
import numpy as np


def nmi(a, b):
    a = np.asarray(a).ravel()
    b = np.asarray(b).ravel()
    if a.size != b.size:
        raise ValueError("label vectors differ in length")
    _, ai = np.unique(a, return_inverse=True)
    _, bi = np.unique(b, return_inverse=True)
    n = a.size
    table = np.zeros((ai.max() + 1, bi.max() + 1))
    np.add.at(table, (ai, bi), 1.0)
    p = table / n
    pa = p.sum(axis=1)
    pb = p.sum(axis=0)
    nz = p > 0
    mi = float(np.sum(p[nz] * (np.log(p[nz]) - np.log(np.outer(pa, pb)[nz]))))
    ha = -float(np.sum(pa[pa > 0] * np.log(pa[pa > 0])))
    hb = -float(np.sum(pb[pb > 0] * np.log(pb[pb > 0])))
    if ha + hb == 0:
        return 1.0
    return mi / (0.5 * (ha + hb))
