// Count arrays, scores and the threshold (Alg. 1; Sec. 3.4.1 Eq. dynadd / dynsub; Sec. 5.3).
//
// Counts are int32 [L][2^K] in device memory, or, with 16-bit counters (the paper's
// short counters, Sec. 3.4), uint16 [L][2^K] that saturate at 65535: an increment of a
// full count is dropped (and counted), a decrement below zero is clamped at zero and
// flagged.  16-bit counts are updated by compare-and-swap on their 32-bit word.
// Alongside the counts the library keeps
// S2_j = sum_b A_j[b]^2 (int64) and S3_j = sum_b A_j[b]^3 (unsigned 128-bit, two
// u64 words), exactly.  An update that moves a count from `old` to `new` adds
// new^2 - old^2 and new^3 - old^3; atomics return `old`, so the deltas telescope to
// the exact sums whatever the order of the updates.  sum_j S2_j / (n L) is the mean
// score of the inserted points (Eq. dynadd / dynsub with the pre-update count).
//
// The scored set keeps m, sum T and sum T^2 (128-bit) exactly in the same way, so
// the threshold's mean and variance come from exact integers.
#include "ace_internal.h"

namespace ace {

namespace {

__device__ inline u64 wave_sum_u64(u64 v) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

__device__ inline void wave_sum_u128(u64& lo, u64& hi) {
    for (int off = 32; off > 0; off >>= 1) {
        const u64 olo = __shfl_xor(lo, off, 64), ohi = __shfl_xor(hi, off, 64);
        const u64 nlo = lo + olo;
        hi = hi + ohi + (nlo < lo ? 1ull : 0ull);
        lo = nlo;
    }
}

__device__ inline void atomic_add_u128(u64* p, u64 lo, u64 hi) {
    const u64 old = atomicAdd(p, lo);
    const u64 carry = (old + lo < old) ? 1ull : 0ull;
    if (hi + carry) atomicAdd(p + 1, hi + carry);
}

// Block-wide sum of (a, b_lo, b_hi) with a 64-bit plain sum and a 128-bit pair; the
// results are valid in thread 0.  `scratch` holds 3 * (blockDim/64) u64.
__device__ inline void block_sum3(u64& a, u64& lo, u64& hi, u64* scratch) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
    a = wave_sum_u64(a);
    wave_sum_u128(lo, hi);
    if (lane == 0) {
        scratch[3 * wave] = a;
        scratch[3 * wave + 1] = lo;
        scratch[3 * wave + 2] = hi;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < nw; ++w) {
            a += scratch[3 * w];
            const u64 nlo = lo + scratch[3 * w + 1];
            hi += scratch[3 * w + 2] + (nlo < lo ? 1ull : 0ull);
            lo = nlo;
        }
    }
}

// Exact change of (count^2, count^3) when a count moves from `old` by `delta`.  Counts
// below 2^21 (cubes below 2^63, the usual case) take 64-bit products.
__device__ inline void sq_cube_delta(int64_t old, int64_t delta, u64& d2, u64& d3lo, u64& d3hi) {
    const int64_t nw64 = old + delta;
    if ((u64)old < ((u64)1 << 21) && (u64)nw64 < ((u64)1 << 21)) {
        const int64_t o2 = old * old, n2 = nw64 * nw64;
        const int64_t dd3 = n2 * nw64 - o2 * old;
        d2 = (u64)(n2 - o2);
        d3lo = (u64)dd3;
        d3hi = dd3 < 0 ? ~0ull : 0ull;
        return;
    }
    const i128 o = old, nw = nw64;
    const i128 dd2 = nw * nw - o * o;
    const i128 dd3 = nw * nw * nw - o * o * o;
    d2 = (u64)(int64_t)dd2;
    const u128 u3 = (u128)dd3;
    d3lo = (u64)u3;
    d3hi = (u64)(u3 >> 64);
}

__device__ inline void add128(u64& lo, u64& hi, u64 alo, u64 ahi) {
    const u64 nlo = lo + alo;
    hi += ahi + (nlo < lo ? 1ull : 0ull);
    lo = nlo;
}

constexpr int HIST_THREADS = 1024;

// Wave-level pre-aggregation of equal buckets.  A bucket held by many lanes of a wave (the
// same code for many rows: duplicated or near-duplicated points) would otherwise take one
// serialised atomic per lane.  The first active lane names its bucket; if at least 16
// lanes hold it, that lane takes all of their updates (a scalar test: one compare and one
// ballot per row, since a fuller search costs more than it saves on ordinary data).
// Returns how many updates this lane applies to its own bucket: the group's size for the
// lane that takes it, 0 for the others of the group, 1 for every other lane.
__device__ inline uint32_t merge_equal_buckets(uint32_t b) {
    const uint32_t lb = __builtin_amdgcn_readfirstlane(b);
    const u64 peers = __ballot(b == lb);
    const uint32_t cnt = (uint32_t)__popcll(peers);
    if (cnt < 16 || b != lb) return 1u;
    const int lane = threadIdx.x & 63;
    return __builtin_amdgcn_readfirstlane(lane) == lane ? cnt : 0u;
}

// Move the 16-bit count b (inside its 32-bit word) by delta: saturate at 65535 going up,
// clamp at 0 (and flag) going down.  Returns the stored value before and after.
__device__ inline void update16(uint32_t* __restrict__ words, int64_t b, int32_t delta, int32_t& before,
                                int32_t& after, unsigned* __restrict__ err) {
    uint32_t* w = words + (b >> 1);
    const int sh = 16 * (int)(b & 1);
    uint32_t cur = __hip_atomic_load(w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    for (;;) {
        const int32_t o = (int32_t)((cur >> sh) & 0xFFFFu);
        int32_t nv = o + delta;
        nv = nv > 65535 ? 65535 : (nv < 0 ? 0 : nv);
        const uint32_t want = (cur & ~(0xFFFFu << sh)) | ((uint32_t)nv << sh);
        const uint32_t prev = atomicCAS(w, cur, want);
        if (prev == cur) {
            before = o;
            after = nv;
            break;
        }
        cur = prev;
    }
    if (delta < 0 && before + delta < 0) atomicOr(err, 1u);
}

// LDS-privatised histogram update of one table over a chunk of rows.
// Grid: (chunks, L).  K <= 15: one uint32 LDS counter per bucket (<= 128 KB).
// K == 16: two uint16 counters per uint32 word (128 KB), chunk <= 65535 rows.
template <bool PACK16, bool C16>
__global__ __launch_bounds__(HIST_THREADS) void update_lds_kernel(const uint16_t* __restrict__ codes, int64_t ldc,
                                                                  int64_t n, int64_t rows_per_block, int K, int sign,
                                                                  void* __restrict__ counts_v, u64* __restrict__ S2,
                                                                  u64* __restrict__ S3, unsigned* __restrict__ err,
                                                                  u64* __restrict__ drops) {
    extern __shared__ uint32_t hist[];
    __shared__ u64 red[3 * (HIST_THREADS / 64)];
    const int j = blockIdx.y;
    const int64_t B = (int64_t)1 << K;
    const int64_t words = PACK16 ? (B >> 1) : B;
    for (int64_t w = threadIdx.x; w < words; w += blockDim.x) hist[w] = 0u;
    __syncthreads();
    const int64_t r0 = (int64_t)blockIdx.x * rows_per_block;
    const int64_t r1 = min(n, r0 + rows_per_block);
    const uint16_t* cj = codes + (int64_t)j * ldc;
    const uint32_t bmask = (uint32_t)(B - 1);  // codes from callers are reduced to K bits
    // Sixteen rows per thread per pass (then four, then one): their codes are all loaded
    // before the first merge test, which needs its row's code in a scalar register, so a
    // pass waits for one round trip to memory instead of one per row.
    auto add = [&](uint32_t b) {
        const uint32_t m = merge_equal_buckets(b);
        if (!m) return;
        if (PACK16)
            atomicAdd(&hist[b >> 1], m << (16 * (b & 1)));
        else
            atomicAdd(&hist[b], m);
    };
    const int64_t bd = blockDim.x;
    int64_t i = r0 + threadIdx.x;
    for (; i + 15 * bd < r1; i += 16 * bd) {
        uint32_t bk[16];
#pragma unroll
        for (int u = 0; u < 16; ++u) bk[u] = cj[i + u * bd] & bmask;
#pragma unroll
        for (int u = 0; u < 16; ++u) add(bk[u]);
    }
    for (; i + 3 * bd < r1; i += 4 * bd) {
        const uint32_t b0 = cj[i] & bmask, b1 = cj[i + bd] & bmask;
        const uint32_t b2 = cj[i + 2 * bd] & bmask, b3 = cj[i + 3 * bd] & bmask;
        add(b0);
        add(b1);
        add(b2);
        add(b3);
    }
    for (; i < r1; i += bd) add(cj[i] & bmask);
    __syncthreads();
    u64 s2 = 0, s3lo = 0, s3hi = 0, dropped = 0;
    auto bucket = [&](int64_t b) -> uint32_t {
        return PACK16 ? ((hist[b >> 1] >> (16 * (b & 1))) & 0xFFFFu) : hist[b];
    };
    if constexpr (C16) {
        for (int64_t b = threadIdx.x; b < B; b += blockDim.x) {
            const uint32_t h = bucket(b);
            if (h) {
                const int32_t delta = sign > 0 ? (int32_t)h : -(int32_t)h;
                int32_t old, nv;
                update16(reinterpret_cast<uint32_t*>(counts_v) + (((int64_t)j * B) >> 1), b, delta, old, nv, err);
                if (sign > 0) dropped += (u64)(delta - (nv - old));
                u64 d2, d3lo, d3hi;
                sq_cube_delta(old, nv - old, d2, d3lo, d3hi);
                s2 += d2;
                add128(s3lo, s3hi, d3lo, d3hi);
            }
        }
    } else {
        // Eight buckets per thread and pass, their returning atomics all issued before the
        // first old value is used (one at a time, each pass would wait a full round trip
        // per bucket).
        constexpr int U = 8;
        int32_t* cnt = reinterpret_cast<int32_t*>(counts_v) + (int64_t)j * B;
        for (int64_t b0 = threadIdx.x; b0 < B; b0 += U * blockDim.x) {
            int32_t delta[U], old[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int64_t b = b0 + u * (int64_t)blockDim.x;
                const uint32_t h = b < B ? bucket(b) : 0u;
                delta[u] = sign > 0 ? (int32_t)h : -(int32_t)h;
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                old[u] = 0;
                if (delta[u] != 0) old[u] = atomicAdd(cnt + b0 + u * (int64_t)blockDim.x, delta[u]);
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                if (delta[u] == 0) continue;
                if ((int64_t)old[u] + delta[u] < 0) atomicOr(err, 1u);
                u64 d2, d3lo, d3hi;
                sq_cube_delta(old[u], delta[u], d2, d3lo, d3hi);
                s2 += d2;
                add128(s3lo, s3hi, d3lo, d3hi);
            }
        }
    }
    if (C16) {
        dropped = wave_sum_u64(dropped);
        if ((threadIdx.x & 63) == 0 && dropped) atomicAdd(drops, dropped);
    }
    block_sum3(s2, s3lo, s3hi, red);
    if (threadIdx.x == 0) {
        if (s2) atomicAdd(&S2[j], s2);
        atomic_add_u128(&S3[2 * j], s3lo, s3hi);
    }
}

// One workgroup per table (K <= 15): the workgroup histograms every row of its table in
// LDS, then moves each bucket once.  It is the only writer of that table during the
// launch, so the counts are read and written plainly (no atomics); the S2/S3 deltas come
// from the old and new value of each bucket, as in the merged kernel.  Grid: L blocks.
template <bool C16>
__global__ __launch_bounds__(HIST_THREADS) void update_table_kernel(const uint16_t* __restrict__ codes, int64_t ldc,
                                                                    int64_t n, int K, int sign,
                                                                    void* __restrict__ counts_v, u64* __restrict__ S2,
                                                                    u64* __restrict__ S3, unsigned* __restrict__ err,
                                                                    u64* __restrict__ drops) {
    extern __shared__ uint32_t hist[];
    __shared__ u64 red[3 * (HIST_THREADS / 64)];
    const int j = blockIdx.x;
    const int64_t B = (int64_t)1 << K;
    for (int64_t w = threadIdx.x; w < B; w += blockDim.x) hist[w] = 0u;
    __syncthreads();
    const uint16_t* cj = codes + (int64_t)j * ldc;
    const uint32_t bmask = (uint32_t)(B - 1);
    auto add = [&](uint32_t b) {
        const uint32_t m = merge_equal_buckets(b);
        if (m) atomicAdd(&hist[b], m);
    };
    const int64_t bd = blockDim.x;
    int64_t i = threadIdx.x;
    for (; i + 15 * bd < n; i += 16 * bd) {   // as in update_lds_kernel
        uint32_t bk[16];
#pragma unroll
        for (int u = 0; u < 16; ++u) bk[u] = cj[i + u * bd] & bmask;
#pragma unroll
        for (int u = 0; u < 16; ++u) add(bk[u]);
    }
    for (; i + 3 * bd < n; i += 4 * bd) {
        const uint32_t b0 = cj[i] & bmask, b1 = cj[i + bd] & bmask;
        const uint32_t b2 = cj[i + 2 * bd] & bmask, b3 = cj[i + 3 * bd] & bmask;
        add(b0);
        add(b1);
        add(b2);
        add(b3);
    }
    for (; i < n; i += bd) add(cj[i] & bmask);
    __syncthreads();
    u64 s2 = 0, s3lo = 0, s3hi = 0, dropped = 0;
    unsigned bad = 0;
    for (int64_t b = threadIdx.x; b < B; b += blockDim.x) {
        const uint32_t h = hist[b];
        if (!h) continue;
        int64_t old, nw;
        if (C16) {
            uint16_t* c = reinterpret_cast<uint16_t*>(counts_v) + (int64_t)j * B + b;
            old = *c;
            nw = sign > 0 ? old + (int64_t)h : old - (int64_t)h;
            if (nw > 65535) {
                dropped += (u64)(nw - 65535);
                nw = 65535;
            }
            if (nw < 0) {
                bad = 1;
                nw = 0;
            }
            *c = (uint16_t)nw;
        } else {
            int32_t* c = reinterpret_cast<int32_t*>(counts_v) + (int64_t)j * B + b;
            old = *c;
            nw = sign > 0 ? old + (int64_t)h : old - (int64_t)h;
            if (nw < 0) bad = 1;
            *c = (int32_t)nw;
        }
        u64 d2, d3lo, d3hi;
        sq_cube_delta(old, nw - old, d2, d3lo, d3hi);
        s2 += d2;
        add128(s3lo, s3hi, d3lo, d3hi);
    }
    if (__any(bad)) {
        if ((threadIdx.x & 63) == 0) atomicOr(err, 1u);
    }
    if (C16) {
        dropped = wave_sum_u64(dropped);
        if ((threadIdx.x & 63) == 0 && dropped) atomicAdd(drops, dropped);
    }
    block_sum3(s2, s3lo, s3hi, red);
    if (threadIdx.x == 0) {
        if (s2) atomicAdd(&S2[j], s2);
        atomic_add_u128(&S3[2 * j], s3lo, s3hi);
    }
}

// Direct update for small batches: one thread per (row, table), one global atomic each.
// Grid: (ceil(n/256), L).
template <bool C16>
__global__ __launch_bounds__(256) void update_direct_kernel(const uint16_t* __restrict__ codes, int64_t ldc,
                                                            int64_t n, int K, int sign, void* __restrict__ counts_v,
                                                            u64* __restrict__ S2, u64* __restrict__ S3,
                                                            unsigned* __restrict__ err, u64* __restrict__ drops) {
    __shared__ u64 red[3 * 4];
    const int j = blockIdx.y;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    u64 s2 = 0, s3lo = 0, s3hi = 0;
    if (i < n) {
        const uint32_t b = codes[(int64_t)j * ldc + i] & ((1u << K) - 1u);
        const uint32_t m = merge_equal_buckets(b);
        if (m) {
            const int32_t delta = sign > 0 ? (int32_t)m : -(int32_t)m;
            int32_t old, moved;
            if (C16) {
                int32_t nv;
                update16(reinterpret_cast<uint32_t*>(counts_v) + (((int64_t)j << K) >> 1), b, delta, old, nv, err);
                moved = nv - old;
                if (sign > 0 && moved != delta) atomicAdd(drops, (u64)(delta - moved));
            } else {
                old = atomicAdd(reinterpret_cast<int32_t*>(counts_v) + ((int64_t)j << K) + b, delta);
                if ((int64_t)old + delta < 0) atomicOr(err, 1u);
                moved = delta;
            }
            sq_cube_delta(old, moved, s2, s3lo, s3hi);
        }
    }
    block_sum3(s2, s3lo, s3hi, red);
    if (threadIdx.x == 0) {
        if (s2) atomicAdd(&S2[j], s2);
        atomic_add_u128(&S3[2 * j], s3lo, s3hi);
    }
}

// A block's (sum T, sum T^2) go to the scored-set moments: straight into mom with atomics,
// or, with mpart, as block b's entry mpart[3 b .. 3 b + 2] for mom_reduce_kernel.  Atomics
// on one address from every block of a large grid are served one after another.
__device__ inline void put_moments(u64 sT, u64 lo, u64 hi, int64_t m, u64* __restrict__ mom,
                                   u64* __restrict__ mpart) {
    if (mpart) {
        mpart[3 * (int64_t)blockIdx.x] = sT;
        mpart[3 * (int64_t)blockIdx.x + 1] = lo;
        mpart[3 * (int64_t)blockIdx.x + 2] = hi;
    } else {
        if (m) atomicAdd(&mom[0], (u64)m);
        atomicAdd(&mom[1], sT);
        atomic_add_u128(&mom[2], lo, hi);
    }
}

// Query phase: T(q) = sum_j A_j[H_j(q)], s = T / L; one thread per row.  The block's
// (m, sum T, sum T^2) are added to the scored-set moments mom[0..3] (put_moments).
template <typename CT>
__global__ __launch_bounds__(256) void score_kernel(const uint16_t* __restrict__ codes, int64_t ldc, int64_t n,
                                                    int K, int L, const CT* __restrict__ counts,
                                                    float* __restrict__ s_out, uint32_t* __restrict__ T_out,
                                                    u64* __restrict__ mom, u64* __restrict__ mpart) {
    __shared__ u64 red[3 * 4];
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    uint32_t T = 0;
    const bool ok = i < n;
    if (ok) {
        const uint16_t* c = codes + i;
        const CT* a = counts;
        const uint32_t bm = (1u << K) - 1u;  // codes from callers are reduced to K bits
        int j = 0;
        for (; j + 4 <= L; j += 4) {
            const uint32_t b0 = c[(int64_t)j * ldc] & bm, b1 = c[(int64_t)(j + 1) * ldc] & bm;
            const uint32_t b2 = c[(int64_t)(j + 2) * ldc] & bm, b3 = c[(int64_t)(j + 3) * ldc] & bm;
            const uint32_t v0 = (uint32_t)a[((int64_t)j << K) + b0];
            const uint32_t v1 = (uint32_t)a[((int64_t)(j + 1) << K) + b1];
            const uint32_t v2 = (uint32_t)a[((int64_t)(j + 2) << K) + b2];
            const uint32_t v3 = (uint32_t)a[((int64_t)(j + 3) << K) + b3];
            T += (v0 + v1) + (v2 + v3);
        }
        for (; j < L; ++j) T += (uint32_t)a[((int64_t)j << K) + (c[(int64_t)j * ldc] & bm)];
        if (s_out) s_out[i] = (float)((double)T / (double)L);
        if (T_out) T_out[i] = T;
    }
    u64 sT = ok ? (u64)T : 0ull;
    const u128 t2 = ok ? (u128)T * (u128)T : (u128)0;
    u64 lo = (u64)t2, hi = (u64)(t2 >> 64);
    block_sum3(sT, lo, hi, red);
    if (threadIdx.x == 0) {
        const int64_t r0 = (int64_t)blockIdx.x * blockDim.x;
        put_moments(sT, lo, hi, min((int64_t)blockDim.x, n - r0), mom, mpart);
    }
}

// Query phase for large batches, table by table: thread g holds rows g and g + G (G threads
// in all) and walks the tables in order, gathering both rows' counts from table j before it
// moves to table j + 1.  Every workgroup then stays near the same table, so the counts it
// gathers are mostly in the L2 of its XCD (connection-log, 6.55 MB of counts: 0.113 against
// 0.130 ms for one row per thread with four tables per step).  Grid: ceil(n / 2) threads.
template <typename CT>
__global__ __launch_bounds__(256) void score_tables_kernel(const uint16_t* __restrict__ codes, int64_t ldc, int64_t n,
                                                           int K, int L, const CT* __restrict__ counts,
                                                           float* __restrict__ s_out, uint32_t* __restrict__ T_out,
                                                           u64* __restrict__ mom, u64* __restrict__ mpart) {
    __shared__ u64 red[3 * 4];
    const int64_t G = (int64_t)gridDim.x * blockDim.x;
    const int64_t i0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x, i1 = i0 + G;
    const bool ok0 = i0 < n, ok1 = i1 < n;
    const uint32_t bm = (1u << K) - 1u;  // codes from callers are reduced to K bits
    uint32_t T0 = 0, T1 = 0;
    for (int j = 0; j < L; ++j) {
        const uint16_t* cj = codes + (int64_t)j * ldc;
        const CT* aj = counts + ((int64_t)j << K);
        const uint32_t b0 = ok0 ? (cj[i0] & bm) : 0u, b1 = ok1 ? (cj[i1] & bm) : 0u;
        if (ok0) T0 += (uint32_t)aj[b0];
        if (ok1) T1 += (uint32_t)aj[b1];
    }
    u64 sT = 0, lo = 0, hi = 0;
    if (ok0) {
        if (s_out) s_out[i0] = (float)((double)T0 / (double)L);
        if (T_out) T_out[i0] = T0;
        sT += T0;
        const u128 t2 = (u128)T0 * (u128)T0;
        add128(lo, hi, (u64)t2, (u64)(t2 >> 64));
    }
    if (ok1) {
        if (s_out) s_out[i1] = (float)((double)T1 / (double)L);
        if (T_out) T_out[i1] = T1;
        sT += T1;
        const u128 t2 = (u128)T1 * (u128)T1;
        add128(lo, hi, (u64)t2, (u64)(t2 >> 64));
    }
    block_sum3(sT, lo, hi, red);
    if (threadIdx.x == 0) put_moments(sT, lo, hi, blockIdx.x == 0 ? n : 0, mom, mpart);
}

// The per-block entries of a score launch (nb of them) summed in one block and added to the
// scored-set moments with the launch's row count m.
__global__ __launch_bounds__(1024) void mom_reduce_kernel(const u64* __restrict__ mpart, int64_t nb, int64_t m,
                                                          u64* __restrict__ mom) {
    __shared__ u64 red[3 * 16];
    u64 sT = 0, lo = 0, hi = 0;
    for (int64_t b = threadIdx.x; b < nb; b += blockDim.x) {
        sT += mpart[3 * b];
        add128(lo, hi, mpart[3 * b + 1], mpart[3 * b + 2]);
    }
    block_sum3(sT, lo, hi, red);
    if (threadIdx.x == 0) {
        atomicAdd(&mom[0], (u64)m);
        atomicAdd(&mom[1], sT);
        atomic_add_u128(&mom[2], lo, hi);
    }
}

// Threshold statistics from the exact sums.
// Unsigned 128-bit integer to the nearest double (ties to even): the top 64 significant
// bits, with a sticky bit for anything below them, go through the correctly rounded u64
// conversion (the sticky bit sits below the rounding position), then an exact scaling.
__device__ inline double u128_to_double(u64 lo, u64 hi) {
    if (hi == 0) return (double)lo;
    const int sh = __clzll((long long)hi);             // 0..63
    const u64 top = sh ? (hi << sh) | (lo >> (64 - sh)) : hi;
    const u64 rest = lo << sh;                          // bits below the top 64 (sh = 0: all of lo)
    return ldexp((double)(top | (rest != 0 ? 1ull : 0ull)), 64 - sh);
}

// One block: thread j takes tables j, j + blockDim, ... (the sum of S2 in 128 bits and the
// per-table deviations), block sums, then thread 0 finishes in FP64.
__global__ __launch_bounds__(256) void threshold_kernel(int64_t n, int L, const u64* __restrict__ S2,
                                                        const u64* __restrict__ S3, const u64* __restrict__ mom,
                                                        const unsigned* __restrict__ err, int mode, double alpha,
                                                        DevThresh* __restrict__ out, double* __restrict__ lim) {
    __shared__ u64 red[3 * 4];
    __shared__ double dsum[4];
    u64 s2lo = 0, s2hi = 0, unused = 0;
    double acc = 0.0;
    for (int j = threadIdx.x; j < L; j += blockDim.x) {
        add128(s2lo, s2hi, S2[j], 0ull);
        if (n > 0) {
            const u128 s3 = ((u128)S3[2 * j + 1] << 64) | S3[2 * j];
            const i128 s2 = (i128)(int64_t)S2[j];
            const i128 v = (i128)n * (i128)s3 - s2 * s2;
            const u128 uv = (u128)v;
            acc += sqrt(u128_to_double((u64)uv, (u64)(uv >> 64))) / (double)n;
        }
    }
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
    if ((threadIdx.x & 63) == 0) dsum[threadIdx.x >> 6] = acc;
    block_sum3(unused, s2lo, s2hi, red);
    if (threadIdx.x != 0) return;
    for (int w = 1; w < (int)(blockDim.x >> 6); ++w) acc += dsum[w];
    DevThresh r;
    r.n = n;
    r.m_scored = (int64_t)mom[0];
    r.mode = mode;
    r.status = 0;
    r.err = err[0];
    r.pad = 0;
    // sum_j S2_j reaches 2^63 well inside the INT32_MAX insert cap (L tables of n^2 each):
    // it is summed and converted in 128 bits.
    r.mu = n > 0 ? u128_to_double(s2lo, s2hi) / ((double)n * (double)L) : 0.0;
    const int64_t m = (int64_t)mom[0];
    const int64_t sumT = (int64_t)mom[1];
    r.mu_scored = 0.0;
    r.sigma = 0.0;
    if (m > 0) {
        const u128 st2 = ((u128)mom[3] << 64) | mom[2];
        const i128 num = (i128)m * (i128)st2 - (i128)sumT * (i128)sumT;
        const u128 un = (u128)num;
        r.mu_scored = (double)sumT / ((double)m * (double)L);
        r.sigma = sqrt(u128_to_double((u64)un, (u64)(un >> 64))) / ((double)m * (double)L);
    }
    r.sigma_table = n > 0 ? acc / (double)L : 0.0;
    r.tau = 0.0;
    if (mode == ACE_THR_SCORED) {
        if (m == 0) r.status = ACE_E_EMPTY;
        else r.tau = r.mu_scored - alpha * r.sigma;
    } else if (mode == ACE_THR_CONST) {
        if (n == 0) r.status = ACE_E_EMPTY;
        else r.tau = r.mu - alpha;
    } else {
        if (n == 0) r.status = ACE_E_EMPTY;
        else r.tau = r.mu - alpha * r.sigma_table;
    }
    *out = r;
    if (lim) *lim = r.status ? __builtin_nan("") : (double)L * r.tau;
}

__global__ __launch_bounds__(256) void flags_kernel(const uint32_t* __restrict__ T, int64_t n, double lim, int le,
                                                    uint8_t* __restrict__ flags) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double t = (double)T[i];
    flags[i] = (uint8_t)(le ? (t <= lim) : (t < lim));
}

// flags_kernel with the limit in device memory (a NaN limit flags nothing).
__global__ __launch_bounds__(256) void flags_dev_kernel(const uint32_t* __restrict__ T, int64_t n,
                                                        const double* __restrict__ lim_p, int le,
                                                        uint8_t* __restrict__ flags) {
    const double lim = *lim_p;   // read before the branch: one scalar load per wave
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double t = (double)T[i];
    flags[i] = (uint8_t)(le ? (t <= lim) : (t < lim));
}

// S2_j and S3_j recomputed from the counts (checkpoint restore).  Grid: L blocks.
template <typename CT>
__global__ __launch_bounds__(256) void table_sums_kernel(const CT* __restrict__ counts, int K,
                                                         u64* __restrict__ S2, u64* __restrict__ S3) {
    __shared__ u64 red[3 * 4];
    const int j = blockIdx.x;
    const int64_t B = (int64_t)1 << K;
    u64 s2 = 0, lo = 0, hi = 0;
    for (int64_t b = threadIdx.x; b < B; b += blockDim.x) {
        const int64_t a = counts[(int64_t)j * B + b];
        s2 += (u64)(a * a);
        const u128 c = (u128)(a * a) * (u128)a;
        add128(lo, hi, (u64)c, (u64)(c >> 64));
    }
    block_sum3(s2, lo, hi, red);
    if (threadIdx.x == 0) {
        S2[j] = s2;
        S3[2 * j] = lo;
        S3[2 * j + 1] = hi;
    }
}

__global__ __launch_bounds__(256) void zero_kernel(uint32_t* __restrict__ p, int64_t words) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < words; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0u;
}

struct ZeroRanges {
    u64* p[4];
    int32_t words[4];   // 64-bit words each
};

// Several small ranges of 64-bit words in one launch (one block; ranges of a few KB).
__global__ __launch_bounds__(256) void zero_ranges_kernel(const ZeroRanges r) {
#pragma unroll
    for (int k = 0; k < 4; ++k)
        for (int i = threadIdx.x; i < r.words[k]; i += blockDim.x) r.p[k][i] = 0ull;
}

}  // namespace

hipError_t init_kernel_attributes() {
    const void* fns[] = {reinterpret_cast<const void*>(&update_table_kernel<false>),
                         reinterpret_cast<const void*>(&update_table_kernel<true>),
                         reinterpret_cast<const void*>(&update_lds_kernel<false, false>),
                         reinterpret_cast<const void*>(&update_lds_kernel<true, false>),
                         reinterpret_cast<const void*>(&update_lds_kernel<false, true>),
                         reinterpret_cast<const void*>(&update_lds_kernel<true, true>)};
    for (const void* f : fns) {
        const hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, 128 * 1024);
        if (e != hipSuccess) return e;
    }
    return init_struct_attributes();
}

hipError_t launch_count_update(const uint16_t* codes, int64_t ldc, int64_t n, int K, int L, int sign,
                               void* counts, int counter_bits, u64* S2, u64* S3, unsigned* err, u64* drops,
                               hipStream_t s) {
    const bool c16 = counter_bits == 16;
    if (n <= 0) return hipSuccess;
    const int64_t B = (int64_t)1 << K;
    // The LDS histogram pays one scan of 2^K buckets per block; use it when a block
    // sees at least 2^K / 2 rows, otherwise one global atomic per (row, table).
    if (n < B / 2) {
        const int64_t nb = (n + 255) / 256;
        if (c16)
            hipLaunchKernelGGL(update_direct_kernel<true>, dim3((unsigned)nb, (unsigned)L), dim3(256), 0, s, codes,
                               ldc, n, K, sign, counts, S2, S3, err, drops);
        else
            hipLaunchKernelGGL(update_direct_kernel<false>, dim3((unsigned)nb, (unsigned)L), dim3(256), 0, s, codes,
                               ldc, n, K, sign, counts, S2, S3, err, drops);
        return hipGetLastError();
    }
    // 16-bit counters, enough tables to fill a good part of the chip and a table that fits
    // in LDS: one workgroup per table (plain stores instead of compare-and-swap loops).
    if (c16 && K <= 15 && L >= 32) {
        const size_t lds = (size_t)B * sizeof(uint32_t);
        if (c16)
            hipLaunchKernelGGL(update_table_kernel<true>, dim3((unsigned)L), dim3(HIST_THREADS), lds, s, codes, ldc,
                               n, K, sign, counts, S2, S3, err, drops);
        else
            hipLaunchKernelGGL(update_table_kernel<false>, dim3((unsigned)L), dim3(HIST_THREADS), lds, s, codes, ldc,
                               n, K, sign, counts, S2, S3, err, drops);
        return hipGetLastError();
    }
    int64_t chunks = (n + B / 2 - 1) / (B / 2);
    // About 256 blocks in total (one per CU): every further chunk of a table adds one
    // returning atomic per non-empty bucket, which costs more than the parallelism buys
    // (connection-log: 0.162 ms with 1024 blocks, 0.097 ms with 256).
    const int64_t want = (256 + L - 1) / L;
    if (chunks > want) chunks = want;
    if (chunks < 1) chunks = 1;
    int64_t rows = (n + chunks - 1) / chunks;
    if (K == 16 && rows > 65535) {
        rows = 65535;
    }
    chunks = (n + rows - 1) / rows;
    const size_t lds = (size_t)(K == 16 ? (B >> 1) : B) * sizeof(uint32_t);
    const dim3 grid((unsigned)chunks, (unsigned)L);
    if (K == 16 && c16)
        hipLaunchKernelGGL((update_lds_kernel<true, true>), grid, dim3(HIST_THREADS), lds, s, codes, ldc, n, rows, K,
                           sign, counts, S2, S3, err, drops);
    else if (K == 16)
        hipLaunchKernelGGL((update_lds_kernel<true, false>), grid, dim3(HIST_THREADS), lds, s, codes, ldc, n, rows, K,
                           sign, counts, S2, S3, err, drops);
    else if (c16)
        hipLaunchKernelGGL((update_lds_kernel<false, true>), grid, dim3(HIST_THREADS), lds, s, codes, ldc, n, rows, K,
                           sign, counts, S2, S3, err, drops);
    else
        hipLaunchKernelGGL((update_lds_kernel<false, false>), grid, dim3(HIST_THREADS), lds, s, codes, ldc, n, rows,
                           K, sign, counts, S2, S3, err, drops);
    return hipGetLastError();
}

hipError_t launch_score(const uint16_t* codes, int64_t ldc, int64_t n, int K, int L, const void* counts,
                        int counter_bits, float* s_out, uint32_t* T_out, u64* mom, hipStream_t s, u64* mpart,
                        int64_t mpart_cap) {
    if (n <= 0) return hipSuccess;
    const bool tables = n >= 131072;   // at least 256 workgroups of the table-by-table kernel
    const int64_t nb = tables ? ((n + 1) / 2 + 255) / 256 : (n + 255) / 256;
    // Past 64 blocks the moments go through per-block entries and one reducing block.
    u64* mp = (mpart && nb > 64 && nb <= mpart_cap) ? mpart : nullptr;
    if (tables) {
        if (counter_bits == 16)
            hipLaunchKernelGGL(score_tables_kernel<uint16_t>, dim3((unsigned)nb), dim3(256), 0, s, codes, ldc, n, K,
                               L, reinterpret_cast<const uint16_t*>(counts), s_out, T_out, mom, mp);
        else
            hipLaunchKernelGGL(score_tables_kernel<int32_t>, dim3((unsigned)nb), dim3(256), 0, s, codes, ldc, n, K, L,
                               reinterpret_cast<const int32_t*>(counts), s_out, T_out, mom, mp);
    } else {
        if (counter_bits == 16)
            hipLaunchKernelGGL(score_kernel<uint16_t>, dim3((unsigned)nb), dim3(256), 0, s, codes, ldc, n, K, L,
                               reinterpret_cast<const uint16_t*>(counts), s_out, T_out, mom, mp);
        else
            hipLaunchKernelGGL(score_kernel<int32_t>, dim3((unsigned)nb), dim3(256), 0, s, codes, ldc, n, K, L,
                               reinterpret_cast<const int32_t*>(counts), s_out, T_out, mom, mp);
    }
    if (!mp) return hipGetLastError();
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(mom_reduce_kernel, dim3(1), dim3(1024), 0, s, mp, nb, n, mom);
    return hipGetLastError();
}

hipError_t launch_threshold(int64_t n, int L, const u64* S2, const u64* S3, const u64* mom, const unsigned* err,
                            int mode, double alpha, DevThresh* out, hipStream_t s, double* lim) {
    hipLaunchKernelGGL(threshold_kernel, dim3(1), dim3(256), 0, s, n, L, S2, S3, mom, err, mode, alpha, out, lim);
    return hipGetLastError();
}

hipError_t launch_flags(const uint32_t* T, int64_t n, int L, double tau, int mode, uint8_t* flags, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    const int64_t nb = (n + 255) / 256;
    hipLaunchKernelGGL(flags_kernel, dim3((unsigned)nb), dim3(256), 0, s, T, n, (double)L * tau,
                       mode == ACE_THR_CONST ? 1 : 0, flags);
    return hipGetLastError();
}

hipError_t launch_flags_dev(const uint32_t* T, int64_t n, const double* lim, int mode, uint8_t* flags, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    const int64_t nb = (n + 255) / 256;
    hipLaunchKernelGGL(flags_dev_kernel, dim3((unsigned)nb), dim3(256), 0, s, T, n, lim, mode == ACE_THR_CONST ? 1 : 0,
                       flags);
    return hipGetLastError();
}

hipError_t launch_table_sums(const void* counts, int counter_bits, int K, int L, u64* S2, u64* S3, hipStream_t s) {
    if (counter_bits == 16)
        hipLaunchKernelGGL(table_sums_kernel<uint16_t>, dim3((unsigned)L), dim3(256), 0, s,
                           reinterpret_cast<const uint16_t*>(counts), K, S2, S3);
    else
        hipLaunchKernelGGL(table_sums_kernel<int32_t>, dim3((unsigned)L), dim3(256), 0, s,
                           reinterpret_cast<const int32_t*>(counts), K, S2, S3);
    return hipGetLastError();
}

// zero_kernel over p, and block 0 also clears the small ranges: one launch for both.
__global__ __launch_bounds__(256) void zero_all_kernel(uint32_t* __restrict__ p, int64_t words, const ZeroRanges r) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < words; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0u;
    if (blockIdx.x != 0) return;
#pragma unroll
    for (int k = 0; k < 4; ++k)
        for (int i = threadIdx.x; i < r.words[k]; i += blockDim.x) r.p[k][i] = 0ull;
}

hipError_t launch_zero_with_small(void* p, size_t bytes, u64* p0, int64_t w0, u64* p1, int64_t w1, u64* p2,
                                  int64_t w2, u64* p3, int64_t w3, hipStream_t s) {
    const int64_t words = (int64_t)(bytes / 4);
    int64_t nb = (words + 255) / 256;
    if (nb > 4096) nb = 4096;
    if (nb < 1) nb = 1;
    ZeroRanges r{{p0, p1, p2, p3}, {(int32_t)w0, (int32_t)w1, (int32_t)w2, (int32_t)w3}};
    hipLaunchKernelGGL(zero_all_kernel, dim3((unsigned)nb), dim3(256), 0, s, reinterpret_cast<uint32_t*>(p), words, r);
    return hipGetLastError();
}

hipError_t launch_zero_small(u64* p0, int64_t w0, u64* p1, int64_t w1, u64* p2, int64_t w2, u64* p3, int64_t w3,
                             hipStream_t s) {
    ZeroRanges r{{p0, p1, p2, p3}, {(int32_t)w0, (int32_t)w1, (int32_t)w2, (int32_t)w3}};
    hipLaunchKernelGGL(zero_ranges_kernel, dim3(1), dim3(256), 0, s, r);
    return hipGetLastError();
}

hipError_t launch_zero(void* p, size_t bytes, hipStream_t s) {
    if (bytes == 0) return hipSuccess;
    const int64_t words = (int64_t)(bytes / 4);
    int64_t nb = (words + 255) / 256;
    if (nb > 4096) nb = 4096;
    hipLaunchKernelGGL(zero_kernel, dim3((unsigned)nb), dim3(256), 0, s, reinterpret_cast<uint32_t*>(p), words);
    return hipGetLastError();
}

}  // namespace ace
