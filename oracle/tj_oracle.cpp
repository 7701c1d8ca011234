// tj_oracle.cpp - CPU oracle for the tensor-path sort and equi-join.
//
// TEST INFRASTRUCTURE ONLY. Nothing on the product path links, loads or calls
// this file; only the test-suite, the smoke check and the CPU-baseline leg of
// the benchmark do. It shares no code, header or table with the GPU library.
//
// Plain, slow, obviously correct definitions, written out directly:
//
//   sort   (tensor-based sort, Sec. IV.B): the stable ascending order of the
//          rows by their key compared as a signed integer. Equal keys keep
//          their input order; the row id travels with its key.
//
//   count  (tensor-based hash join, Sec. IV.A): the size of the inner equi-join
//          on the key attribute, |R join S| = sum over keys k of
//          cnt_R(k) * cnt_S(k), as an unsigned 64-bit number.
//
//   pairs  (Sec. IV.A with late materialisation, Sec. III.A): every matching
//          (rid_R[i], rid_S[j]) with key_R[i] == key_S[j], emitted in the
//          canonical order: ascending key, then R input position, then S input
//          position (R-major within a key).
//
// The paper fixes neither the sort direction, stability, key signedness nor
// the order of join output; the readings above are the ones the GPU library
// guarantees.
//
// Library primitives used as single steps: std::sort (with a total order on
// (key, position), which makes the result unique) and std::unordered_map.
// Parity pinned by: brute-force nested loops and insertion sort on tiny inputs,
// numpy's stable argsort, closed-form join sizes built into the generators, and
// the invariants (sorted, permutation, stability, sum cnt_R*cnt_S).

#include <algorithm>
#include <cstdint>
#include <cstring>
#include <unordered_map>
#include <vector>

namespace {

template <typename K>
void oracle_sort(const K* keys, const int32_t* rids, uint64_t n, K* keys_out, int32_t* rids_out)
{
    std::vector<uint64_t> idx(n);
    for (uint64_t i = 0; i < n; i++) idx[i] = i;
    // Strict total order on (key, input position): the stable order.
    std::sort(idx.begin(), idx.end(), [keys](uint64_t a, uint64_t b) {
        return keys[a] < keys[b] || (keys[a] == keys[b] && a < b);
    });
    for (uint64_t i = 0; i < n; i++) {
        keys_out[i] = keys[idx[i]];
        rids_out[i] = rids[idx[i]];
    }
}

template <typename K>
uint64_t oracle_join_count(const K* r_keys, uint64_t n_r, const K* s_keys, uint64_t n_s)
{
    std::unordered_map<K, uint64_t> cnt_r;
    cnt_r.reserve(n_r);
    for (uint64_t i = 0; i < n_r; i++) cnt_r[r_keys[i]] += 1;
    // Probing S row by row adds cnt_R(k) once per S row with key k, which sums
    // to cnt_R(k) * cnt_S(k) per key.
    uint64_t total = 0;
    for (uint64_t j = 0; j < n_s; j++) {
        auto it = cnt_r.find(s_keys[j]);
        if (it != cnt_r.end()) total += it->second;
    }
    return total;
}

// Writes the first min(count, capacity) pairs of the canonical order and
// returns count.
template <typename K>
uint64_t oracle_join_pairs(const K* r_keys, const int32_t* r_rids, uint64_t n_r,
                           const K* s_keys, const int32_t* s_rids, uint64_t n_s,
                           int32_t* out_r, int32_t* out_s, uint64_t capacity)
{
    struct Lists {
        std::vector<uint64_t> r, s;
    };
    std::unordered_map<K, Lists> by_key;
    by_key.reserve(n_r);
    for (uint64_t i = 0; i < n_r; i++) by_key[r_keys[i]].r.push_back(i);  // R positions, input order
    std::vector<K> matched;
    for (uint64_t j = 0; j < n_s; j++) {
        auto it = by_key.find(s_keys[j]);
        if (it == by_key.end()) continue;
        if (it->second.s.empty()) matched.push_back(s_keys[j]);
        it->second.s.push_back(j);  // S positions, input order
    }
    std::sort(matched.begin(), matched.end());  // ascending key
    uint64_t t = 0;
    for (K k : matched) {
        const Lists& l = by_key[k];
        for (uint64_t i : l.r)
            for (uint64_t j : l.s) {
                if (t < capacity) {
                    out_r[t] = r_rids[i];
                    out_s[t] = s_rids[j];
                }
                t++;
            }
    }
    return t;
}

// All pairs with key == k, in canonical order, by two linear scans.
template <typename K>
uint64_t oracle_pairs_for_key(K k, const K* r_keys, const int32_t* r_rids, uint64_t n_r,
                              const K* s_keys, const int32_t* s_rids, uint64_t n_s,
                              int32_t* out_r, int32_t* out_s, uint64_t capacity)
{
    std::vector<uint64_t> rs, ss;
    for (uint64_t i = 0; i < n_r; i++)
        if (r_keys[i] == k) rs.push_back(i);
    for (uint64_t j = 0; j < n_s; j++)
        if (s_keys[j] == k) ss.push_back(j);
    uint64_t t = 0;
    for (uint64_t i : rs)
        for (uint64_t j : ss) {
            if (t < capacity) {
                out_r[t] = r_rids[i];
                out_s[t] = s_rids[j];
            }
            t++;
        }
    return t;
}

}  // namespace

extern "C" {

void tjo_sort_i32(const int32_t* k, const int32_t* r, uint64_t n, int32_t* ko, int32_t* ro)
{
    oracle_sort<int32_t>(k, r, n, ko, ro);
}

void tjo_sort_i64(const int64_t* k, const int32_t* r, uint64_t n, int64_t* ko, int32_t* ro)
{
    oracle_sort<int64_t>(k, r, n, ko, ro);
}

uint64_t tjo_join_count_i32(const int32_t* kr, uint64_t nr, const int32_t* ks, uint64_t ns)
{
    return oracle_join_count<int32_t>(kr, nr, ks, ns);
}

uint64_t tjo_join_count_i64(const int64_t* kr, uint64_t nr, const int64_t* ks, uint64_t ns)
{
    return oracle_join_count<int64_t>(kr, nr, ks, ns);
}

uint64_t tjo_join_pairs_i32(const int32_t* kr, const int32_t* rr, uint64_t nr, const int32_t* ks,
                            const int32_t* rs, uint64_t ns, int32_t* out_r, int32_t* out_s,
                            uint64_t cap)
{
    return oracle_join_pairs<int32_t>(kr, rr, nr, ks, rs, ns, out_r, out_s, cap);
}

uint64_t tjo_join_pairs_i64(const int64_t* kr, const int32_t* rr, uint64_t nr, const int64_t* ks,
                            const int32_t* rs, uint64_t ns, int32_t* out_r, int32_t* out_s,
                            uint64_t cap)
{
    return oracle_join_pairs<int64_t>(kr, rr, nr, ks, rs, ns, out_r, out_s, cap);
}

uint64_t tjo_pairs_for_key_i32(int32_t k, const int32_t* kr, const int32_t* rr, uint64_t nr,
                               const int32_t* ks, const int32_t* rs, uint64_t ns, int32_t* out_r,
                               int32_t* out_s, uint64_t cap)
{
    return oracle_pairs_for_key<int32_t>(k, kr, rr, nr, ks, rs, ns, out_r, out_s, cap);
}

uint64_t tjo_pairs_for_key_i64(int64_t k, const int64_t* kr, const int32_t* rr, uint64_t nr,
                               const int64_t* ks, const int32_t* rs, uint64_t ns, int32_t* out_r,
                               int32_t* out_s, uint64_t cap)
{
    return oracle_pairs_for_key<int64_t>(k, kr, rr, nr, ks, rs, ns, out_r, out_s, cap);
}

}  // extern "C"
