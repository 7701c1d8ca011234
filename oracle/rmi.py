"""CPU oracle of the learned CDF partitioner (test infrastructure).

Only the test-suite, the smoke check and the benchmark's CPU-baseline leg use
this module; it shares no code with the GPU library.

The partitioner replaces the radix digit of the first partition pass by a
bucket function learned from a sample of the keys: a two-layer recursive model
index (RMI) whose first layer is a piecewise-linear map over equal-depth knots
of the sorted sample and whose second layer is 1024 linear models, each fitted
by least squares to the sample points routed to it.  The method keeps its
results exact for any bucket function that is non-decreasing in the key (the
rows of bucket b then all precede those of bucket b + 1 in key order), so the
function is built to be monotone: non-negative slopes, and each leaf's output
clamped to a bucket interval that never overlaps the next leaf's.

The paper leaves the data characteristics to be used at execution time open
(Sec. III.C: the path is chosen and tuned from what the execution stage
observes); this model is that observation, made on a sample.

Definition followed here, step by step (every float operation is the one the
device evaluates, in the same precision, so bucket ids are reproducible bit
for bit from the same model):

  ordinal:  ord(k) = k XOR 2^63 as uint64 (int64 keys), (k XOR 2^31) as uint32
            (int32 keys): an order-preserving map to unsigned integers.
  sample:   a relation of n rows gives m = max(min(n, 2048), floor(n * permille
            / 1000)) rows at positions floor(i * n / m), i < m; a join samples
            both relations and fits one model to the union.
  sort:     the union's ordinals ascending: s[0 .. M).
  root:     knot[i] = s[floor(i (M - 1) / 256)], i = 0 .. 256;
            inv[i] = f32(1 / f64(knot[i+1] - knot[i])), 0 when the two knots are
            equal. For a key x: j = the largest i in [0, 255] with i = 0 or
            knot[i] <= x; d = clamp(x, knot[j], knot[j+1]) - knot[j];
            t = f32(d) * inv[j] (f32); leaf = 4 j + min(floor(4 t), 3).
  leaves:   sample point i with leaf l gets target y_i = F i / M (F = buckets);
            leaf l's points are a contiguous run [a, b) of s. base = s[a];
            d_i = f64(s_i - base); slope = max(0, S_dy / S_dd) (0 when S_dd = 0),
            with the centred sums S_dd = sum (d_i - mean d)^2 and
            S_dy = sum (d_i - mean d)(y_i - mean y); intercept = mean y -
            slope * mean d; both stored as f32. lo = floor(F a / M),
            hi = floor(F (b - 1) / M). A leaf without points takes
            base = 0, slope = intercept = 0, lo = hi = lo of the next leaf that
            has points (F - 1 when none follows).
  bucket:   l = leaf(x); sd = x - base_l as a signed integer saturated to
            +-2^62; y = a_l + b_l * f32(sd) (two f32 roundings, no fused
            multiply-add); bucket = floor(clamp(y, lo_l, hi_l)).
Parity note: the integer fields (knots, bases, lo, hi) and inv are exactly
reproducible; slope and intercept come from fp64 sums whose order differs
between implementations, so they agree to a few f32 ulps.
"""
from __future__ import annotations

import numpy as np

SEGMENTS = 256
LEAVES = 1024
SUB = LEAVES // SEGMENTS
SAT = 1 << 62


def ordinals(keys: np.ndarray) -> np.ndarray:
    """Order-preserving map of signed keys to uint64 ordinals."""
    if keys.dtype == np.int64:
        return keys.view(np.uint64) ^ np.uint64(1 << 63)
    if keys.dtype == np.int32:
        return (keys.view(np.uint32) ^ np.uint32(1 << 31)).astype(np.uint64)
    raise TypeError(keys.dtype)


def sample_count(n: int, permille: int) -> int:
    return max(min(n, 2048), n * permille // 1000)


def sample_positions(n: int, permille: int) -> np.ndarray:
    m = sample_count(n, permille)
    # i * n < 2^62 for n < 2^31: exact in uint64
    return ((np.arange(m, dtype=np.uint64) * np.uint64(n)) // np.uint64(m)).astype(np.int64)


def u64_to_f32(v: np.ndarray) -> np.ndarray:
    """Round non-negative integers (< 2^64) to the nearest float32, ties to even,
    with integer arithmetic only (no float64 intermediate)."""
    v = np.asarray(v, dtype=np.uint64)
    out = np.empty(v.shape, dtype=np.float32)
    small = v < np.uint64(1 << 24)
    out[small] = v[small].astype(np.float32)  # exact
    big = ~small
    if big.any():
        x = v[big]
        # bit length
        nb = np.zeros(x.shape, dtype=np.int64)
        t = x.copy()
        for s in (32, 16, 8, 4, 2, 1):
            m = t >= np.uint64(1 << s)
            nb[m] += s
            t[m] >>= np.uint64(s)
        nb += 1
        sh = (nb - 24).astype(np.uint64)
        q = x >> sh
        rem = x - (q << sh)
        half = np.uint64(1) << (sh - np.uint64(1))
        up = (rem > half) | ((rem == half) & ((q & np.uint64(1)) == np.uint64(1)))
        q = q + up.astype(np.uint64)
        # q * 2^sh is exact in float64 (q <= 2^24), and then exact in float32
        out[big] = (q.astype(np.float64) * np.exp2(sh.astype(np.float64))).astype(np.float32)
    return out


def i64_to_f32(v: np.ndarray) -> np.ndarray:
    v = np.asarray(v, dtype=np.int64)
    neg = v < 0
    mag = np.where(neg, -v, v).astype(np.uint64)  # |v| <= 2^62 here
    f = u64_to_f32(mag)
    return np.where(neg, -f, f).astype(np.float32)


class Model:
    """The fitted parameters (host arrays); field names follow the C header."""

    def __init__(self, F: int):
        self.buckets = F
        self.sample_rows = 0
        self.knot = np.zeros(SEGMENTS + 1, dtype=np.uint64)
        self.knot_inv = np.zeros(SEGMENTS, dtype=np.float32)
        self.leaf_base = np.zeros(LEAVES, dtype=np.uint64)
        self.leaf_a = np.zeros(LEAVES, dtype=np.float32)
        self.leaf_b = np.zeros(LEAVES, dtype=np.float32)
        self.leaf_lo = np.zeros(LEAVES, dtype=np.uint16)
        self.leaf_hi = np.zeros(LEAVES, dtype=np.uint16)


def root_leaf(model: Model, x: np.ndarray) -> np.ndarray:
    """First layer: leaf index of each ordinal x."""
    x = np.asarray(x, dtype=np.uint64)
    kn = model.knot
    # largest i in [0, 255] with i == 0 or knot[i] <= x
    j = np.searchsorted(kn[1:SEGMENTS], x, side="right").astype(np.int64)
    lo = kn[j]
    hi = kn[j + 1]
    xc = np.minimum(np.maximum(x, lo), hi)
    d = xc - lo
    t = (u64_to_f32(d) * model.knot_inv[j]).astype(np.float32)
    q = (t * np.float32(SUB)).astype(np.float32)
    sub = np.where(q >= np.float32(SUB - 1), SUB - 1, np.floor(q)).astype(np.int64)
    return j * SUB + sub


def bucket(model: Model, x: np.ndarray) -> np.ndarray:
    """The learned bucket function on ordinals x (uint64 array)."""
    x = np.asarray(x, dtype=np.uint64)
    leaf = root_leaf(model, x)
    base = model.leaf_base[leaf]
    ge = x >= base
    pos = np.minimum(np.where(ge, x - base, 0), np.uint64(SAT)).astype(np.int64)
    neg = np.minimum(np.where(ge, 0, base - x), np.uint64(SAT)).astype(np.int64)
    sd = pos - neg
    prod = (model.leaf_b[leaf] * i64_to_f32(sd)).astype(np.float32)
    y = (model.leaf_a[leaf] + prod).astype(np.float32)
    lo = model.leaf_lo[leaf].astype(np.float32)
    hi = model.leaf_hi[leaf].astype(np.float32)
    y = np.where(y < lo, lo, np.where(y > hi, hi, y))
    return np.floor(y).astype(np.int64)


def train(key_arrays, buckets: int = 512, permille: int = 10) -> Model:
    """Fit the model to the sample of each key array (one array: sort; two: join)."""
    parts = []
    for k in key_arrays:
        n = len(k)
        if n == 0:
            continue
        parts.append(ordinals(np.asarray(k))[sample_positions(n, permille)])
    s = np.sort(np.concatenate(parts)) if parts else np.zeros(1, dtype=np.uint64)
    M = len(s)
    F = buckets
    m = Model(F)
    m.sample_rows = M
    idx = (np.arange(SEGMENTS + 1, dtype=np.int64) * (M - 1)) // SEGMENTS
    m.knot[:] = s[idx]
    D = m.knot[1:] - m.knot[:-1]
    with np.errstate(divide="ignore"):
        m.knot_inv[:] = np.where(D > 0, (1.0 / D.astype(np.float64)), 0.0).astype(np.float32)
    # the float64 conversion of D above is the f64(D) of the definition: exact
    # below 2^53 and correctly rounded above, as on the device
    leaf = root_leaf(m, s)
    starts = np.searchsorted(leaf, np.arange(LEAVES + 1), side="left")
    y_all = float(F) * np.arange(M, dtype=np.float64) / float(M)
    nonempty = np.zeros(LEAVES, dtype=bool)
    for l in range(LEAVES):
        a, b = int(starts[l]), int(starts[l + 1])
        if b <= a:
            continue
        nonempty[l] = True
        base = s[a]
        d = (s[a:b] - base).astype(np.float64)
        y = y_all[a:b]
        dm, ym = d.mean(), y.mean()
        sdd = float(((d - dm) ** 2).sum())
        sdy = float(((d - dm) * (y - ym)).sum())
        slope = max(0.0, sdy / sdd) if sdd > 0 else 0.0
        m.leaf_base[l] = base
        m.leaf_b[l] = np.float32(slope)
        m.leaf_a[l] = np.float32(ym - slope * dm)
        m.leaf_lo[l] = (F * a) // M
        m.leaf_hi[l] = (F * (b - 1)) // M
    nxt = F - 1
    for l in range(LEAVES - 1, -1, -1):
        if nonempty[l]:
            nxt = int(m.leaf_lo[l])
        else:
            m.leaf_lo[l] = m.leaf_hi[l] = nxt
    return m
