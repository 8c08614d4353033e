"""||U^T U - I||_F of a large device matrix U, exactly up to the final rounding, with torch's
FP64 matrix product (rocBLAS / hipBLASLt) -- independent of the library under test.

Each column j of U is written as 2^e_j x_j with |x_j| < 1 (e_j from the column maximum),
and x_j * 2^72 is cut into four signed 18-bit integer pieces (entries below 2^(e_j - 72) are
dropped: an error under 2^-72 of the column's largest entry).  A product of two pieces has at
most 36 bits, so the sum of such products over a chunk of 2^16 rows stays below 2^52: the FP64
GEMM of two piece matrices is then exact whatever its summation order.  The piece pairs
(a, b) with a + b <= 3 are formed (the others weigh below 2^-72 relative), summed over the
chunks in int64, and combined with their power-of-two scales in double-double on the host.
"""
from __future__ import annotations

import numpy as np

CHUNK = 1 << 16
PIECES = 4
BITS = 18


def _two_sum(a, b):
    s = a + b
    bv = s - a
    return s, (a - (s - bv)) + (b - bv)


def gram_exact(U) -> tuple[np.ndarray, np.ndarray]:
    """U^T U of a column-major FP64 torch CUDA matrix as a double-double (hi, lo) pair of
    numpy arrays."""
    import torch
    m, n = int(U.shape[0]), int(U.shape[1])
    amax = U.abs().amax(dim=0)
    e = torch.where(amax > 0, torch.frexp(amax)[1], torch.zeros_like(amax, dtype=torch.int32))
    e = e.to(torch.int64)  # 2^(e - 1) <= max |u| < 2^e
    acc = {}
    pairs = [(a, b) for a in range(PIECES) for b in range(PIECES) if a + b <= PIECES - 1]
    scale = torch.ldexp(torch.ones(n, dtype=torch.float64, device=U.device),
                        (PIECES * BITS - e).to(torch.float64))
    for r0 in range(0, m, CHUNK):
        blk = U[r0:r0 + CHUNK]
        X = torch.trunc(blk * scale[None, :])  # |X| < 2^72, an integer (exact: power-of-two scale)
        pieces = []
        rest = X
        for a in range(PIECES):
            w = 2.0 ** (BITS * (PIECES - 1 - a))
            p = torch.trunc(rest / w)
            pieces.append(p.contiguous())
            rest = rest - p * w
        for (a, b) in pairs:
            P = (pieces[a].t() @ pieces[b]).to(torch.int64)
            acc[(a, b)] = acc[(a, b)] + P if (a, b) in acc else P
    ecpu = e.cpu().numpy()
    hi = np.zeros((n, n))
    lo = np.zeros((n, n))
    base = ecpu[:, None] + ecpu[None, :] - 2 * PIECES * BITS
    for (a, b), P in acc.items():
        Pn = P.cpu().numpy()
        ph = Pn.astype(np.float64)
        pl = (Pn - ph.astype(np.int64)).astype(np.float64)  # exact remainder
        sh = np.ldexp(1.0, base + BITS * ((PIECES - 1 - a) + (PIECES - 1 - b)))
        th, tl = ph * sh, pl * sh  # exact scalings by powers of two
        s, err = _two_sum(hi, th)
        hi, lo = s, lo + err + tl
    hi, lo = _two_sum(hi, lo)
    return hi, lo


def orth_exact(U) -> float:
    """||U^T U - I||_F with U^T U exact to double-double rounding."""
    hi, lo = gram_exact(U)
    n = hi.shape[0]
    d = (hi - np.eye(n)) + lo
    return float(np.linalg.norm(d))
