"""Low-rank compression of admissible blocks (oracle).

Section 2.3.2 ("SVD-based low-rank compression"): an admissible block B (p' x q')
at one lag is replaced by U_k Sigma_k V_k^T, keeping the singular values above a
tolerance; when k is not much smaller than min(p', q') the factors would cost
more than the block, and the block is kept dense.  The paper's tolerance is an
absolute threshold on singular values; ``relative=True`` scales it by the
largest singular value (the library's ACA uses a relative Frobenius criterion).
"""
from __future__ import annotations

import numpy as np


def truncated_svd(B, tol, relative=False):
    U, s, Vt = np.linalg.svd(B, full_matrices=False)
    thr = tol * (s[0] if (relative and s.size) else 1.0)
    k = int(np.sum(s > thr))
    return U[:, :k] * s[:k], Vt[:k].T, k


def stored_entries(p, q, k):
    """Entries kept for a block of rank k: k (p + q) if that is less than p q."""
    return min(k * (p + q), p * q)
