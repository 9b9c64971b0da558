"""Accuracy of the split-f16 exponent of the FP32 / BF16 matrix-core products,
emulated on the CPU with numpy float16 (no GPU, no library code).

The kernel forms the folded exponent arg = 2 t . o + c (c = -|t|^2 - N_J) as an
inner product of f16 slots: every FP32 operand v is split into hi = f16(v) and
lo = f16(v - hi), each coordinate contributes o_hi 2t_hi + o_hi 2t_lo + o_lo 2t_hi
(the lo * lo term is dropped) and the constant contributes c_hi + c_lo.  The
products are exact in the FP32 accumulator.  These tests pin the error of that
representation: the bound per operand, the exponent error on tiles at the fold
limit, and the figure at the largest operands a folded tile admits.
"""
import numpy as np

F16, F32 = np.float16, np.float32
FOLD_R2 = 40.0   # squared tile radius (scaled units) above which the direct form is used


def split(v):
    v = F32(v)
    hi = F16(v)
    return hi, F16(F32(v) - F32(hi))


def split_exponent(t2, o, c):
    """The slot inner product (in FP64, so only the representation error shows)."""
    s = 0.0
    for tk, ok in zip(t2, o):
        th, tl = split(tk)
        oh, ol = split(ok)
        s += float(oh) * float(th) + float(oh) * float(tl) + float(ol) * float(th)
    ch, cl = split(c)
    return s + float(ch) + float(cl)


def test_split_representation_bound():
    # |v - hi - lo| <= 2^-22 |v| + 2^-25 (half an f16 subnormal step) over
    # magnitudes from the f16 subnormal range to the largest folded operands;
    # the bound is reached within a factor of two, so 2^-24 would be wrong
    rng = np.random.default_rng(0)
    v = (rng.choice([-1.0, 1.0], 200_000) * 10.0 ** rng.uniform(-6, 2.9, 200_000)).astype(np.float32)
    hi = v.astype(np.float16)
    lo = (v - hi.astype(np.float32)).astype(np.float16)
    err = np.abs(v.astype(np.float64) - hi.astype(np.float64) - lo.astype(np.float64))
    bound = 2.0 ** -22 * np.abs(v.astype(np.float64)) + 2.0 ** -25
    assert np.all(err <= bound)
    assert (err / np.abs(v.astype(np.float64))).max() > 2.0 ** -23


def test_exponent_error_at_fold_limit():
    # targets and sources anywhere on a tile of squared radius R^2 = 40 (2-D and
    # 3-D), with the tile's normaliser N_J = floor(R^2 / 2): the emulated
    # exponent against the exact one of the same FP32 operands stays within the
    # analytic bound 3 * 2^-22 * sum_k |2 t_k o_k| + 2^-22 |c| (+ subnormal
    # steps), and within 6e-5 in absolute terms; for the pairs whose kernel
    # value matters (distance below 4 bandwidth-scaled units) the relative
    # kernel error ln2 * |d arg| stays below 2e-5
    rng = np.random.default_rng(1)
    R = np.sqrt(FOLD_R2)
    nj = np.floor(FOLD_R2 / 2)
    worst, worst_near = 0.0, 0.0
    for d in (2, 3):
        for _ in range(20_000):
            o = rng.normal(size=d)
            o *= R * rng.uniform(0.5, 1.0) / np.linalg.norm(o)
            t = o + rng.normal(scale=rng.choice([0.3, 1.0, 3.0]), size=d)
            t2 = (2.0 * t.astype(np.float32)).astype(np.float32)
            o32 = o.astype(np.float32)
            tt = float(np.dot(t.astype(np.float32).astype(np.float64), t.astype(np.float32).astype(np.float64)))
            c = F32(-F32(tt) - F32(nj))
            exact = float(np.dot(t2.astype(np.float64), o32.astype(np.float64))) + float(c)
            err = abs(split_exponent(t2, o32, c) - exact)
            bound = 3 * 2.0 ** -22 * float(np.abs(t2.astype(np.float64) * o32).sum()) + 2.0 ** -22 * abs(float(c)) \
                + 6 * 2.0 ** -25 * (float(np.abs(t2).sum() + np.abs(o32).sum()) + 1.0)
            assert err <= bound
            worst = max(worst, err)
            if np.linalg.norm(t - o) < 4.0:
                worst_near = max(worst_near, np.log(2.0) * err)
    assert worst <= 6e-5, worst
    assert worst_near <= 2e-5, worst_near


def test_exponent_error_at_largest_folded_operands():
    # the largest operands a folded tile admits before the far clamp, as quoted
    # for R^2 = 64: |2t| ~ 29, |o| ~ 8, |c| ~ 240 (a target at the edge of the
    # contributing range).  The exponent error reaches about 6e-5 there, but the
    # kernel value of such a pair is below 2^-20 (squared distance above 20
    # scaled units), so the absolute error it adds is below 1e-10 of the self
    # pair's value; at the current fold limit (R^2 <= 40) these operands shrink
    # to |o| <= 6.3
    rng = np.random.default_rng(2)
    errs = []
    for _ in range(5000):
        u = rng.normal(size=2)
        u /= np.linalg.norm(u)
        o = (8.0 * u).astype(np.float32)
        t = 14.5 * u + rng.normal(scale=0.5, size=2)
        t2 = (2.0 * t).astype(np.float32)
        c = F32(-240.0 + rng.uniform(-1, 1))
        exact = float(np.dot(t2.astype(np.float64), o.astype(np.float64))) + float(c)
        errs.append(abs(split_exponent(t2, o, c) - exact))
        dist2 = float(np.dot(t - o, t - o))
        assert dist2 > 20.0  # kernel value 2^-dist2 < 2^-20
    assert 1e-5 < max(errs) < 1.2e-4
