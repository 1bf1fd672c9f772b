"""The reduced chain of the mixed form above K = 8, on the host: with the
three-piece BF16 split (each piece the round-to-nearest-even BF16 of the
remainder left by the previous ones, so piece i is at most 2^-8i of the
value), the products it leaves out (pieces of order 2 for coefficients
8..11, of order 1 and 2 for 12..15) change a position by at most
0.99 ((3 + 2^-7) 2^-25 + (2^-7 (1 + 2^-8) + 3.01 * 2^-16) 2^-17), about
2.49 * 2^-24, of the template's contraction bound whenever that template's
group bounds meet the limits the kernel tests (group 2 at most 0.99 * 2^-9,
group 3 at most 0.99 * 2^-17 of the sum over all groups); with three groups
(K = 9 .. 12) the group-2 term alone, about 1.49 * 2^-24.  The full chains
themselves accumulate up to 18 or 24 products in FP32, each addition
rounding by up to 2^-24 of its partial sum."""

LIMIT2 = 0.99 * (3 + 2.0 ** -7) * 2.0 ** -25
LIMIT = LIMIT2 + 0.99 * (2.0 ** -7 * (1 + 2.0 ** -8) + 3.01 * 2.0 ** -16) * 2.0 ** -17
import numpy as np
import pytest


def bf16_rne(x):
    """FP32 -> nearest BF16 (ties to even), returned as FP32."""
    b = np.asarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    b = (b + 0x7FFF + ((b >> 16) & 1)) & 0xFFFF0000
    return b.astype(np.uint32).view(np.float32)


def split3(x64):
    """Three BF16 pieces of an FP64 value, each from the FP64 remainder."""
    p0 = bf16_rne(np.float32(x64)).astype(np.float64)
    r1 = x64 - p0
    p1 = bf16_rne(np.float32(r1)).astype(np.float64)
    p2 = bf16_rne(np.float32(r1 - p1)).astype(np.float64)
    return p0, p1, p2


def test_piece_magnitudes():
    g = np.random.default_rng(5)
    x = g.standard_normal(200000) * np.exp(g.uniform(-30, 30, 200000))
    p0, p1, p2 = split3(x)
    assert np.all(np.abs(p1) <= np.abs(x) * 2.0 ** -8)
    assert np.all(np.abs(p2) <= np.abs(x) * 2.0 ** -16)
    # the three pieces carry the value to 24 bits
    assert np.all(np.abs(x - p0 - p1 - p2) <= np.abs(x) * 2.0 ** -24)


@pytest.mark.parametrize("K", [16, 12])
def test_left_out_products_within_bound(K):
    g = np.random.default_rng(6 + K)
    n = 20000
    limit = LIMIT if K > 12 else LIMIT2
    worst = 0.0
    for trial in range(4):
        u = g.standard_normal((n, K)) * 300.0              # U[alpha, k] T of one segment, per draw
        c = g.uniform(-3, 3, (n, K)).astype(np.float32).astype(np.float64)
        mag = np.abs(c) * np.abs(u)
        # scale groups 2 and 3 to the limits (and a random share below them)
        allg = mag[:, :8].sum(1)
        s2 = g.uniform(0.2, 1.0, n) * 0.99 * 2.0 ** -9
        s3 = g.uniform(0.2, 1.0, n) * 0.99 * 2.0 ** -17 if K > 12 else np.zeros(n)
        # choose the group sums so that bg2 = s2 * all and bg3 = s3 * all
        # with all = bg0 + bg1 + bg2 + bg3
        tot = allg / (1.0 - s2 - s3)
        u[:, 8:12] *= (s2 * tot / mag[:, 8:12].sum(1))[:, None]
        if K > 12:
            u[:, 12:16] *= (s3 * tot / mag[:, 12:16].sum(1))[:, None]
        cf = c.astype(np.float32)
        cp = [bf16_rne(cf).astype(np.float64)]
        cp.append(bf16_rne((cf - cp[0].astype(np.float32)).astype(np.float32)).astype(np.float64))
        cp.append(bf16_rne((cf - cp[0].astype(np.float32) - cp[1].astype(np.float32)).astype(np.float32))
                  .astype(np.float64))
        up = split3(u)
        order2 = cp[1] * up[1] + cp[0] * up[2] + cp[2] * up[0]
        order1 = cp[0] * up[1] + cp[1] * up[0]
        left_out = order2[:, 8:12].sum(1) + (order1 + order2)[:, 12:16].sum(1)   # empty above K
        bound = (np.abs(cf.astype(np.float64)) * np.abs(u)).sum(1)
        r = np.abs(left_out) / bound
        worst = max(worst, float(r.max()))
    assert LIMIT < 2.5 * 2.0 ** -24 and LIMIT2 < 1.5 * 2.0 ** -24
    assert worst <= limit, worst
    # the bound is reached only when every piece sits at its largest
    # remainder; random draws stay well inside it
    assert worst >= limit / 16, worst
