"""Helpers of the GPU tests: error norms of a state against the oracle."""
import numpy as np

FAMILIES = {"rho": [0], "m": [1, 2, 3], "e": [4], "b": [5, 6, 7]}


def family_rel_err(a, b):
    """max |a - b| / max |b| over each field family (rho, m, e, b)."""
    out = {}
    for k, idx in FAMILIES.items():
        den = np.abs(b[idx]).max()
        out[k] = float(np.abs(a[idx] - b[idx]).max() / den) if den > 0 else float(np.abs(a[idx]).max())
    return out


def l1_rel(a, b):
    """mean over fields of mean|a-b| / mean|b|; a field with zero reference
    uses the scale of its family."""
    errs = []
    for k, idx in FAMILIES.items():
        fam = np.mean(np.abs(b[idx]))
        for f in idx:
            den = np.mean(np.abs(b[f]))
            if den == 0:
                den = fam if fam > 0 else 1.0
            errs.append(np.mean(np.abs(a[f] - b[f])) / den)
    return float(np.mean(errs))


def max_family_err(a, b):
    return max(family_rel_err(a, b).values())
