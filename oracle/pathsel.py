"""CPU oracle of the execution-time path selection (test infrastructure).

Only the test-suite, the smoke check and the benchmark's CPU-baseline leg use
this module; it shares no code with the GPU library.

The paper chooses, at execution time and per operation, between the existing
linear (CPU) path and the tensor path from indicators that are cheap to
observe then: the scale of the inputs, the cardinality of the join attribute
and the expected size of the intermediate result (Sec. III.C; the effect of
the choice is measured in Sec. V.D). The paper leaves the estimators and the
thresholds open; the reading followed here:

  hash:      h(k) = the SplitMix64 output function (Steele, Lea, Flood 2014)
             applied to (k + 0x9E3779B97F4A7C15) mod 2^64, k the key as a
             signed 64-bit integer (int32 keys sign-extended); h(k) is the
             first output of a SplitMix64 generator seeded with k.
  registers: HyperLogLog (Flajolet, Fusy, Gandouet, Meunier 2007) with
             m = 2^14 registers; key k goes to register j = h >> 50 with rank
             rho = 1 + (number of leading zeros of the low 50 bits of h, read
             as a 50-bit word), or 51 when they are all zero; M[j] = largest
             rank seen, 0 if none.
  estimate:  Z = sum_j 2^-M[j]; E = alpha_m m^2 / Z with alpha_m = 0.7213 /
             (1 + 1.079 / m); if E <= 5 m / 2 and V = #{j : M[j] = 0} > 0,
             E = m ln(m / V) (linear counting). Z is summed exactly, as the
             integer sum_j 2^(51 - M[j]), and divided once in float64.
  union:     registers max(M_R[j], M_S[j]) (the sketch of R union S).
  common:    d_common = max(0, min(d_R, d_S, d_R + d_S - d_union)).
  output:    d_common * (n_R / d_R) * (n_S / d_S): rows spread evenly over
             each side's distinct keys (0 when a side is empty).
  decision:  tensor when n_R + n_S >= min_rows, or (join) when the expected
             output >= min_output; otherwise linear.
"""
import math

import numpy as np

M_BITS = 14
M = 1 << M_BITS
MAX_RANK = 64 - M_BITS + 1
GAMMA = 0x9E3779B97F4A7C15
DEFAULT_MIN_ROWS = 1 << 11
DEFAULT_MIN_OUTPUT = 1 << 10
_MASK = (1 << 64) - 1


def hash64(keys):
    """SplitMix64 output for the state key + gamma, elementwise (uint64)."""
    with np.errstate(over="ignore"):
        z = np.asarray(keys).astype(np.int64).view(np.uint64) + np.uint64(GAMMA)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        return z ^ (z >> np.uint64(31))


def hash64_scalar(k):
    """The same hash in Python integers, for single keys."""
    z = (int(k) + GAMMA) & _MASK
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _MASK
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _MASK
    return z ^ (z >> 31)


def index_rank(h):
    """Register index and rank of hash values h (uint64 array)."""
    h = np.asarray(h, dtype=np.uint64)
    idx = (h >> np.uint64(64 - M_BITS)).astype(np.int64)
    low = h & np.uint64((1 << (64 - M_BITS)) - 1)
    # rank = 1 + leading zeros of `low` as a 50-bit word = 50 - bit_length(low) + 1;
    # low < 2^53 converts to float64 exactly, and frexp's exponent of a positive
    # x is its bit length (frexp(0) gives 0)
    bl = np.frexp(low.astype(np.float64))[1].astype(np.int64)
    rank = (64 - M_BITS) - bl + 1
    return idx, rank.astype(np.uint8)


def registers(keys):
    """HyperLogLog registers (uint8[M]) of a key column."""
    reg = np.zeros(M, dtype=np.uint8)
    keys = np.asarray(keys)
    if keys.size == 0:
        return reg
    for a in range(0, keys.size, 1 << 24):  # in slices, to bound the temporaries
        idx, rank = index_rank(hash64(keys[a:a + (1 << 24)]))
        np.maximum.at(reg, idx, rank)
    return reg


def estimate(reg):
    """The HyperLogLog cardinality estimate of registers `reg`."""
    reg = np.asarray(reg)
    z = 0
    for r, c in enumerate(np.bincount(reg.astype(np.int64), minlength=MAX_RANK + 1)):
        z += int(c) << (MAX_RANK - r)
    m = float(M)
    alpha = 0.7213 / (1.0 + 1.079 / m)
    e = alpha * m * m * 2.0 ** MAX_RANK / float(z)
    v = int(np.count_nonzero(reg == 0))
    if e <= 2.5 * m and v > 0:
        e = m * math.log(m / float(v))
    return e


def select(r_keys, s_keys=None, min_rows=0, min_output=0):
    """The selection of one sort (s_keys None) or join: a dict of the
    indicators, the decision and the three register arrays."""
    min_rows = min_rows or DEFAULT_MIN_ROWS
    min_output = min_output or DEFAULT_MIN_OUTPUT
    join = s_keys is not None
    r_keys = np.asarray(r_keys)
    s_keys = np.asarray(s_keys if join else r_keys[:0])
    reg_r = registers(r_keys)
    reg_s = registers(s_keys)
    reg_u = np.maximum(reg_r, reg_s)
    n_r, n_s = int(r_keys.size), int(s_keys.size)
    d_r = estimate(reg_r)
    d_s = estimate(reg_s) if join else 0.0
    d_u = estimate(reg_u)
    common = est = 0.0
    if join:
        common = max(0.0, min(d_r, d_s, d_r + d_s - d_u))
        if d_r > 0 and d_s > 0:
            est = common * (n_r / d_r) * (n_s / d_s)
    reasons = (1 if n_r + n_s >= min_rows else 0) | (2 if join and est >= min_output else 0)
    return {"n_r": n_r, "n_s": n_s, "distinct_r": d_r, "distinct_s": d_s, "distinct_union": d_u,
            "distinct_common": common, "est_output": est, "path": 1 if reasons else 0, "reasons": reasons,
            "registers": np.stack([reg_r, reg_s, reg_u])}
