"""Element-wise comparison of the MLP kernels with the float64 reference.

Both sides round the same values to bfloat16 at the same points, so every
output element is a sum of the same bfloat16 products, summed in float32 on
the GPU and in float64 by the reference.  Measured against the element's
term scale S (the sum of the absolute values of its terms, from
mlp_ref.term_scales):
  - with identical factors the two sums differ by at most (K-1) 2^-24 S for
    K terms (float32 accumulation), below 1e-3 S for any K here;
  - a factor whose float32 and float64 values straddle a bfloat16 rounding
    midpoint is rounded one ulp apart on the two sides (at most 2^-7 of its
    magnitude; this happens to roughly one rounded value in 10^4), which can
    move an element it enters by up to 2^-7 of that term.
So an element may leave the 1e-3 S band only through such a flip: at most a
small counted fraction of a block may, and none by more than 2^-6 S (two
flipped factors in one term).
"""
import numpy as np

TIGHT = 1e-3
LOOSE = 2.0 ** -6
MAX_OUTLIER_FRAC = 0.005

# parameter blocks of the 8705-vector: W1, b1, W2, b2, W3, b3, W4, b4
BLOCKS = [("W1", 0, 256), ("b1", 256, 320), ("W2", 320, 4416), ("b2", 4416, 4480), ("W3", 4480, 8576),
          ("b3", 8576, 8640), ("W4", 8640, 8704), ("b4", 8704, 8705)]


def compare(got, want, scale):
    """(ok, worst error over scale, number of elements beyond TIGHT)."""
    got, want, scale = (np.asarray(a, np.float64) for a in (got, want, scale))
    e = np.abs(got - want) / np.maximum(scale, 1e-300)
    n_out = int(np.count_nonzero(e > TIGHT))
    ok = bool(e.max() <= LOOSE) and n_out <= int(MAX_OUTLIER_FRAC * e.size)
    return ok, float(e.max()), n_out


def compare_grad(got, want, scale):
    """compare() per parameter block; returns (all ok, {block: result})."""
    res = {name: compare(got[a:b], want[a:b], scale[a:b]) for name, a, b in BLOCKS}
    return all(r[0] for r in res.values()), res
