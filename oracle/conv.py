"""Oracle (test infrastructure only): 2-D convolution from its definition.

Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
import this module; the product path never does.

The Stream-K chapter's conclusion names convolution among the GEMM-like
problems the decomposition extends to.  A convolution is the GEMM whose A is
the input gathered per output pixel (implicit GEMM); the result oracle is the
convolution itself, written from its definition in float64:

  y[n, p, q, k] = alpha * sum_{r, s, c} x[n, p*u + r*dh - ph, q*v + s*dw - pw, c] * w[k, r, s, c]
                  + beta * y_in[n, p, q, k]

with x NHWC, w KRSC, y NPQK (channels innermost), zero for input positions
outside the image (padding), P = (H + 2 ph - dh (R - 1) - 1) // u + 1 and Q
likewise.  The sum over the R x S window is taken tap by tap; each tap is one
float64 contraction over the channels (a library matrix product as a step).
Its GEMM view, which the schedule of a convolution follows: M = N P Q output
pixels (n, then p, then q), N = K output channels, and the reduction index
kk = (r S + s) C + c.
"""
from __future__ import annotations

import numpy as np


def out_size(H, W, R, S, ph, pw, u, v, dh, dw):
    P = (H + 2 * ph - dh * (R - 1) - 1) // u + 1
    Q = (W + 2 * pw - dw * (S - 1) - 1) // v + 1
    return P, Q


def conv2d_f64(x, w, pad=(0, 0), stride=(1, 1), dil=(1, 1), alpha=1.0, beta=0.0, y=None):
    """The definition above, in float64.  x: N x H x W x C, w: K x R x S x C."""
    x = np.asarray(x, dtype=np.float64)
    w = np.asarray(w, dtype=np.float64)
    N, H, W_, C = x.shape
    K, R, S, C2 = w.shape
    assert C == C2
    ph, pw = pad
    u, v = stride
    dh, dw = dil
    P, Q = out_size(H, W_, R, S, ph, pw, u, v, dh, dw)
    xp = np.zeros((N, H + 2 * ph, W_ + 2 * pw, C))
    xp[:, ph:ph + H, pw:pw + W_, :] = x
    acc = np.zeros((N, P, Q, K))
    for r in range(R):
        for s in range(S):
            h0, w0 = r * dh, s * dw
            tap = xp[:, h0:h0 + (P - 1) * u + 1:u, w0:w0 + (Q - 1) * v + 1:v, :]   # N x P x Q x C
            acc += tap @ w[:, r, s, :].T
    out = alpha * acc
    if beta != 0.0:
        out = out + beta * np.asarray(y, dtype=np.float64)
    return out


def conv2d_loops(x, w, pad=(0, 0), stride=(1, 1), dil=(1, 1)):
    """The same definition as pure Python loops (for tiny cases only)."""
    N, H, W_, C = x.shape
    K, R, S, _ = w.shape
    P, Q = out_size(H, W_, R, S, pad[0], pad[1], stride[0], stride[1], dil[0], dil[1])
    y = np.zeros((N, P, Q, K))
    for n in range(N):
        for p in range(P):
            for q in range(Q):
                for k in range(K):
                    t = 0.0
                    for r in range(R):
                        for s in range(S):
                            h = p * stride[0] + r * dil[0] - pad[0]
                            ww = q * stride[1] + s * dil[1] - pad[1]
                            if 0 <= h < H and 0 <= ww < W_:
                                for c in range(C):
                                    t += float(x[n, h, ww, c]) * float(w[k, r, s, c])
                    y[n, p, q, k] = t
    return y
