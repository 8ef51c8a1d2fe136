"""Element-wise and block-wise error bounds for the reduced-precision sweeps.

A sweep in FP32 or BF16 rounds each core value once (unit roundoff u of the
compute type), the FP64 input once when the first core reads it, and each
stored intermediate y_k once; every core's products are summed in FP32
(K_in = r_{k-1} n_k terms, unit roundoff 2^-24 per addition at worst).  Each
of these is a relative perturbation of one factor of the product of the cores
(the TT definition, section 2.2), so the computed Y satisfies, entry by entry,

    |Y - A X| <= ((1 + u)^(2d) (1 + 2^-24)^(sum_k K_in,k) - 1) (|A| |X|),

where |A| is the QTT matrix with cores |G_k| (the magnitude of every term of
the sum that defines A(i, j)) and |X| the entrywise magnitude.  The oracle
applies |A| to |X| in FP64.  A small absolute floor covers FP32 underflow.

"fp32s" is the FP32 sweep with products formed from split BF16 operands
(v = bf16(v) + bf16(v - bf16(v)) + e, |e| <= 2^-16 |v|, the product of the
two lo parts omitted): each product term is off by at most
(1 + 2^-24)^2 (1 + 2^-16)^2 - 1 + 2^-16 (1 + 2^-8)^2 < 4 * 2^-16 of its
size, covered by two factors (1 + 2^-15) per core; its three matrix
instructions per contraction index triple the FP32 additions.
"""
import numpy as np

from oracle import qtt_oracle as O

UNIT = {"fp32": 2.0 ** -24, "bf16": 2.0 ** -8, "fp32s": 2.0 ** -15}
ACC_TERMS = {"fp32": 1, "bf16": 1, "fp32s": 3}
U_ACC = 2.0 ** -24


def growth(cores, dtype):
    d = len(cores)
    kin = sum(G.shape[0] * G.shape[2] for G in cores)
    return (1.0 + UNIT[dtype]) ** (2 * d) * (1.0 + U_ACC) ** (ACC_TERMS[dtype] * kin) - 1.0


def magnitude(cores, X):
    """|A| |X| by the oracle (FP64)."""
    return O.qtt_apply_alg2([np.abs(G) for G in cores], np.abs(np.asarray(X)))


def elementwise_ratio(Y, ref, cores, X, dtype, mag=None):
    """max_i |Y - ref|_i / bound_i (<= 1 means the bound holds everywhere)."""
    Y = np.asarray(Y).reshape(ref.shape)
    if mag is None:
        mag = magnitude(cores, X).reshape(ref.shape)
    bound = growth(cores, dtype) * mag + 1e-30 * max(float(np.abs(ref).max()), 1e-300)
    return float(np.max(np.abs(Y - ref) / bound))


def blockwise_rel(Y, ref, rows=512):
    """Largest relative error over blocks of `rows` consecutive entries of any
    column: a wrong tile shows up in the blocks it touches even when the
    column's norm hides it."""
    Y = np.asarray(Y).reshape(ref.shape[0], -1)
    R = ref.reshape(ref.shape[0], -1)
    worst = 0.0
    for c in range(R.shape[1]):
        for r0 in range(0, R.shape[0], rows):
            num = np.linalg.norm(Y[r0:r0 + rows, c] - R[r0:r0 + rows, c])
            den = np.linalg.norm(R[r0:r0 + rows, c])
            if den > 0:
                worst = max(worst, num / den)
            elif num > 0:
                worst = np.inf
    return worst
