"""Discrete trigonometric transforms attached to boundary symmetries.

Paper, Section 3.2.2: Table 2 maps the pair of symmetries of a nodal field on
the two faces of an axis to a transform (SS -> DCT1, SA -> DCT3, AA -> DST1,
AS -> DST3; periodic -> DFT); Table 3 and eq (7) state that each transform
coefficient equals, up to a factor alpha, one selected coefficient of the DFT
of the 4n-periodic symmetric extension of the signal.

Reading of Table 3 (its DST rows are garbled in the extracted text): the
selected real-space nodes S_R and the angle theta of each coefficient are

    DCT1  nodes 0..n      theta_m = pi m / n,        m = 0..n      alpha = 2
    DCT3  nodes 0..n-1    theta_m = pi (m + 1/2)/n,  m = 0..n-1    alpha = 2
    DST1  nodes 1..n-1    theta_m = pi m / n,        m = 1..n-1    alpha = -2i
    DST3  nodes 1..n      theta_m = pi (m + 1/2)/n,  m = 0..n-1    alpha = -2i
    DFT   nodes 0..n-1    theta_k = 2 pi k / n (real half-complex storage)

Forward transforms are unnormalised; the inverse of a DTT of type T is the
"transpose" transform divided by 2n (DCT1 -> DCT1, DCT3 -> DCT2, DST1 -> DST1,
DST3 -> DST2), and the inverse DFT is divided by n.  The normalisation alpha
of eq (7) does not change the Green solve, since the same factor appears in
the forward and the inverse step.

Two implementations live here: `forward_matrix`/`inverse_matrix` write the
defining sums out (O(n^2), used on small sizes and as a pin), and
`forward`/`inverse` call scipy.fft (a library primitive) for speed.  Tests
pin both against each other, against round trips, and against numpy's DFT of
the explicit 4n extension (eq 7).
"""
from __future__ import annotations

import numpy as np
import scipy.fft as sfft

TYPES = ("DCT1", "DCT3", "DST1", "DST3", "DFT")

# Table 2 (nodal fields): symmetry on face 0 and face 1 -> transform
SYM_TO_TYPE = {("S", "S"): "DCT1", ("S", "A"): "DCT3", ("A", "A"): "DST1",
               ("A", "S"): "DST3", ("P", "P"): "DFT"}


def selection(kind, n):
    """Real-space node indices S_R (Table 3) for an axis of n voxels."""
    return {"DCT1": np.arange(0, n + 1), "DCT3": np.arange(0, n),
            "DST1": np.arange(1, n), "DST3": np.arange(1, n + 1),
            "DFT": np.arange(0, n)}[kind]


def thetas(kind, n):
    """Angle theta of every stored coefficient, in storage order."""
    if kind == "DCT1":
        return np.pi * np.arange(0, n + 1) / n
    if kind == "DST1":
        return np.pi * np.arange(1, n) / n
    if kind in ("DCT3", "DST3"):
        return np.pi * (np.arange(0, n) + 0.5) / n
    if kind == "DFT":
        k = np.arange(n)
        k = np.minimum(k, n - k)        # half-complex slot k and n-k hold frequency min(k, n-k)
        return 2.0 * np.pi * k / n
    raise ValueError(kind)


def _ends_weight(idx, lo, hi):
    w = np.full(idx.shape, 2.0)
    w[(idx == lo) | (idx == hi)] = 1.0
    return w


def forward_matrix(kind, n):
    """Defining sums of the forward transform: X_m = sum_k w_k x_k phi(theta_m k),
    with w_k = 1 for the end nodes 0 and n and 2 otherwise (each interior node
    appears twice in one period of the symmetric extension)."""
    if kind == "DFT":
        k = np.arange(n)
        F = np.zeros((n, n))
        for m in range(n):
            if m <= n // 2:
                F[m] = np.cos(2 * np.pi * m * k / n)
            else:
                F[m] = -np.sin(2 * np.pi * (n - m) * k / n)
        return F
    k = selection(kind, n)
    th = thetas(kind, n)
    w = _ends_weight(k, 0, n)
    phi = np.cos if kind.startswith("DCT") else np.sin
    return phi(np.outer(th, k)) * w[None, :]


def inverse_matrix(kind, n):
    """Defining sums of the inverse: x_k = (1/2n) sum_m v_m X_m phi(theta_m k), with
    v_m = 1 where theta_m is 0 or pi and 2 otherwise (1/n and half-complex for DFT)."""
    if kind == "DFT":
        return np.linalg.inv(forward_matrix(kind, n))
    k = selection(kind, n)
    th = thetas(kind, n)
    v = np.full(th.shape, 2.0)
    v[np.isclose(th, 0.0) | np.isclose(th, np.pi)] = 1.0
    phi = np.cos if kind.startswith("DCT") else np.sin
    return phi(np.outer(k, th)) * v[None, :] / (2.0 * n)


def forward(x, kind, axis, n):
    """Forward transform along `axis` of the already-selected samples (scipy.fft)."""
    if kind == "DCT1":
        return sfft.dct(x, type=1, axis=axis)
    if kind == "DCT3":
        return sfft.dct(x, type=3, axis=axis)
    if kind == "DST1":
        return sfft.dst(x, type=1, axis=axis)
    if kind == "DST3":
        return sfft.dst(x, type=3, axis=axis)
    if kind == "DFT":
        X = np.moveaxis(sfft.rfft(x, axis=axis), axis, -1)
        out = np.empty(X.shape[:-1] + (n,))
        h = n // 2
        out[..., :h + 1] = X.real[..., :h + 1]
        for k in range(1, (n + 1) // 2):
            out[..., n - k] = X.imag[..., k]
        return np.moveaxis(out, -1, axis)
    raise ValueError(kind)


def inverse(X, kind, axis, n):
    """Inverse transform along `axis` (scipy.fft), back to the selected samples."""
    if kind == "DCT1":
        return sfft.dct(X, type=1, axis=axis) / (2.0 * n)
    if kind == "DCT3":
        return sfft.dct(X, type=2, axis=axis) / (2.0 * n)
    if kind == "DST1":
        return sfft.dst(X, type=1, axis=axis) / (2.0 * n)
    if kind == "DST3":
        return sfft.dst(X, type=2, axis=axis) / (2.0 * n)
    if kind == "DFT":
        Xm = np.moveaxis(X, axis, -1)
        h = n // 2
        C = np.zeros(Xm.shape[:-1] + (h + 1,), dtype=np.complex128)
        C.real[...] = Xm[..., :h + 1]
        for k in range(1, (n + 1) // 2):
            C.imag[..., k] = Xm[..., n - k]
        return np.moveaxis(sfft.irfft(C, n=n, axis=-1), -1, axis)
    raise ValueError(kind)


def extension_4n(q, kind, n):
    """Build the 4n-periodic extension q4 of a nodal line q[0..n] with the
    symmetries of `kind` (S: even, A: odd) about x=0 and x=n (Section 3.2.2).

    The reflection about 0 gives q(-x) = s0 q(x) and the one about n gives
    q(n+y) = s1 q(n-y); together q(x + 2n) = s0 s1 q(x)."""
    s0, s1 = {"DCT1": (1, 1), "DCT3": (1, -1), "DST1": (-1, -1), "DST3": (-1, 1)}[kind]
    q = np.asarray(q, dtype=np.float64).copy()
    if s0 < 0:
        q[0] = 0.0
    if s1 < 0:
        q[n] = 0.0
    out = np.empty(4 * n)
    for j in range(4 * n):
        t, r = divmod(j, 2 * n)
        v = q[r] if r <= n else s1 * q[2 * n - r]
        out[j] = v * (s0 * s1) ** t
    return out


def s4f(kind, n):
    """Selection S_4F of eq (7): indices in the 4n-point DFT, and the factor alpha."""
    if kind == "DCT1":
        return 2 * np.arange(0, n + 1), 2.0
    if kind == "DCT3":
        return 2 * np.arange(0, n) + 1, 2.0
    if kind == "DST1":
        return 2 * np.arange(1, n), -2.0j
    if kind == "DST3":
        return 2 * np.arange(0, n) + 1, -2.0j
    raise ValueError(kind)
