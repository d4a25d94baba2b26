// SRP hashing on BF16 MFMA with split operands (Sec. 2.1 signed random projections,
// Sec. 3.2 K-bit codes), v_mfma_f32_16x16x32_bf16, FP32 accumulate.
//
// Every FP32 input is split exactly into x = x_h + x_l + rho_x with x_h = bf16(x),
// x_l = bf16(x - x_h) (round to nearest even) and rho_x = x - x_h - x_l (exact in
// FP32); W likewise, ahead of time.  The kernel accumulates two chains on the
// matrix unit:
//     main = sum_t x_h w_h          corr = sum_t (x_h w_l + x_l w_h)
// and takes p~ = main + corr.  The remainder p - (S_hh + S_hl + S_lh) is
//     sum_t (x_h rho_w + x_l w_l + x_l rho_w + rho_x w),
// bounded by Cauchy-Schwarz.  Accumulation error of a chain of I instructions is at
// most hm u sum|products| (main) and hc u sum|products| (corrections), u = 2^-23:
//   measured model (gfx950 probes: the 8 products of a k-group are aligned to the
//   group's largest and cut below 2^-24 of it; group sums enter the accumulator with
//   round-to-nearest): hm = 4 + 2 I, hc = 4 + 4 I;
//   generic model (an instruction may lose 34 units relative to |acc| + sum|p|):
//   hm = 34 I, hc = 68 I.
// Hence, with A = ||x_h||, B = ||x_l||, C = ||rho_x||:
//     |p - p~| <= A cA_c + B cB_c + C cC_c + eps_c
//     cA = ||rho_w|| + hm u ||w_h|| + hc u ||w_l|| + 2u (||w_h|| + ||w_l||)
//     cB = ||w_l|| + ||rho_w|| + hc u ||w_h|| + 2u ||w_h||
//     cC = ||w||
// (I = padded d / 32; eps_c covers flushed subnormal products), all rounded up by
// the host.  Outside the bound the sign of p~ is the sign of p; inside it the
// projection is queued for the FP64 pass, exactly as in the FP32 kernel.
//
// Tiling: 256 threads = 4 waves as 2 (rows) x 2 (columns); workgroup tile 128 rows
// x 2*TW tables (TW <= 4); per wave 64 rows x TW tables, 2 x 4 x TW accumulators of
// 16x16.  The register budget (256 per lane) keeps two waves per SIMD, and two
// workgroups (64 KB of LDS each) share a CU.  X is split into hi/lo once per chunk by
// convert_bf16_kernel (which also writes the three row norms) into 16 x 32 tiles of
// 1 KB (bf16_tiled_index); W's split is stored the same way.  Each k-step of 32 then
// moves whole tiles from global memory straight into LDS (one 16-byte load per lane,
// no registers in between), into one of two stages, while the MFMAs read the other.
//
// Where the time goes (low-rank 1M x 1024 launch): the MFMAs alone take 2.9 ms and the
// tile loads alone 3.8 ms; together 5.5 ms.  The loads, not the matrix unit, bound the
// kernel: per k, a 128 x 128 tile loads 1 KB of split operands for 3 x 128 x 128
// products (96 FLOP per byte), and two accumulator chains leave no registers for a
// larger tile.
#include <type_traits>

#include "ace_internal.h"

namespace ace {

namespace {

constexpr int BM = 128;
constexpr int BK = 32;

typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef short s4v __attribute__((ext_vector_type(4)));

// Sign packing.  Lane l stores row rho = l & 15 of 16-row tile l >> 4.  Tile b's ballot of
// accumulator element r holds row 4g + r in bits 16g .. 16g + 15 (lane 16g + c holds column
// c), so lane l needs ballot pick = 4 (l >> 4) + (l & 3) shifted right by 16 ((l & 15) >> 2).
// f[e] is ballot e already shifted by the lane's amount; a select tree over the bits of pick
// keeps the lane's own (masks, not branches or a switch).
__device__ inline uint32_t pick_code(uint32_t (&f)[16], int pick) {
#pragma unroll
    for (int w = 1; w < 16; w <<= 1) {
        const uint32_t m = 0u - (uint32_t)((pick & w) != 0);
#pragma unroll
        for (int i = 0; i + w < 16; i += 2 * w) f[i] = (f[i + w] & m) | (f[i] & ~m);
    }
    return f[0];
}

__device__ inline uint32_t wave_sum_u32(uint32_t v) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Round-to-nearest-even FP32 -> BF16 bits, and back.  Inputs are finite.
__device__ inline uint16_t bf16_bits(float x) {
    uint32_t u = __float_as_uint(x);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
__device__ inline float bf16_val(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

// Convert + row norms: X (FP32 [n][d]) -> Xh, Xl (bf16 bits in 16 x 32 tiles, zero-padded
// to DP and to whole 16-row tiles) and the row norms A = ||x_h||, B = ||x_l||,
// C = ||rho_x|| (FP32 sums of squares rounded up by norm_up, square roots by 2^-20).
// LPR lanes per row (64 for rows of 256 or more k, fewer for short rows, so that no lane
// idles): lane l of a row takes the 4 consecutive k at 4l + 4 LPR i and writes 8 bytes of
// hi and 8 of lo.
template <bool VEC, int LPR>
__global__ __launch_bounds__(256) void convert_bf16_kernel(const float* __restrict__ X, int64_t n, int64_t n16, int d, int DP,
                                                           uint16_t* __restrict__ Xh, uint16_t* __restrict__ Xl,
                                                           float* __restrict__ rowA, float* __restrict__ rowB,
                                                           float* __restrict__ rowC, float norm_up) {
    constexpr int RPW = 64 / LPR;  // rows per wave
    const int lane = threadIdx.x & (LPR - 1);
    const int64_t row = ((int64_t)blockIdx.x * 4 + (threadIdx.x >> 6)) * RPW + (threadIdx.x & 63) / LPR;
    if (row >= n16) return;        // a row's LPR lanes leave together
    const bool real = row < n;  // rows n .. n16-1 fill the last 16-row tile with zeros
    const float* xr = X + (real ? row : 0) * (int64_t)d;
    float sA = 0.f, sB = 0.f, sC = 0.f;
    for (int k0 = 4 * lane; k0 < DP; k0 += 4 * LPR) {
        f4 v;
        if (!real) {
            v = f4{0.f, 0.f, 0.f, 0.f};
        } else if (VEC && k0 + 4 <= d) {
            v = __builtin_nontemporal_load(reinterpret_cast<const f4*>(xr + k0));
        } else {
#pragma unroll
            for (int e = 0; e < 4; ++e) v[e] = (k0 + e < d) ? xr[k0 + e] : 0.f;
        }
        s4v ph, pl;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const uint16_t hb = bf16_bits(v[e]);
            const float hv = bf16_val(hb);
            const float r1 = v[e] - hv;  // exact
            const uint16_t lb = bf16_bits(r1);
            const float lv = bf16_val(lb);
            const float r2 = r1 - lv;    // exact
            sA = fmaf(hv, hv, sA);
            sB = fmaf(lv, lv, sB);
            sC = fmaf(r2, r2, sC);
            ph[e] = (short)hb;
            pl[e] = (short)lb;
        }
        // Plain stores: a row fills half of each 128-byte line of a tile and the next row
        // (another wave of the block) the other half; the cache merges them (nontemporal
        // stores of the halves took 15.6 against 13.3 ms per low-rank step).
        const size_t o = bf16_tiled_index(row, k0, DP);
        *reinterpret_cast<s4v*>(Xh + o) = ph;
        *reinterpret_cast<s4v*>(Xl + o) = pl;
    }
    if (!real) return;
    for (int off = LPR / 2; off > 0; off >>= 1) {  // within the row's lanes
        sA += __shfl_xor(sA, off, 64);
        sB += __shfl_xor(sB, off, 64);
        sC += __shfl_xor(sC, off, 64);
    }
    if (lane == 0) {
        rowA[row] = sqrtf(sA * norm_up) * (1.f + 0x1p-20f);
        rowB[row] = sqrtf(sB * norm_up) * (1.f + 0x1p-20f);
        rowC[row] = sqrtf(sC * norm_up) * (1.f + 0x1p-20f);
    }
}

// The tile layout's chunk rotation (tile_chunk_swz) keeps the fragment reads (16 rows x
// one chunk per quarter-wave) free of LDS bank conflicts on gfx950, as 96-byte padded
// rows would (measured with SQ_LDS_BANK_CONFLICT; plain 64-byte rows, and rotations by
// r & 3 or (r >> 2) & 3, conflict two-way), while a tile row stays 64 bytes.

// One wave-wide 16-byte-per-lane load from global memory straight into LDS: lane l's
// 16 bytes land at lds + 16 l (lds is the same for every lane).
__device__ inline void load_to_lds16(const uint16_t* g, char* lds) {
    __builtin_amdgcn_global_load_lds(g, (__attribute__((address_space(3))) void*)lds, 16, 0, 0);
}

// Wait until this wave's loads into LDS have landed.
__device__ inline void wait_lds_loads() { asm volatile("s_waitcnt vmcnt(0)" ::: "memory"); }

template <int TW>
__global__ __launch_bounds__(256, 2) void hash_bf16_kernel(const HashArgs a) {
    constexpr int NB = 32 * TW;
    constexpr int A_BYTES = BM * 2 * BK;               // one of x_h / x_l per stage (8 KB)
    constexpr int B_BYTES = NB * 2 * BK;               // one of w_h / w_l per stage
    constexpr int STAGE = 2 * A_BYTES + 2 * B_BYTES;
    constexpr int NI = STAGE / 1024;                   // 1 KB wave loads per stage (16 + 4 TW)
    constexpr int PW = NI / 4;                         // per wave
    static_assert(NI % 4 == 0, "stage loads split evenly over the four waves");
    __shared__ __attribute__((aligned(1024))) char st0[STAGE];
    __shared__ __attribute__((aligned(1024))) char st1[STAGE];

    const int64_t bid = blockIdx.x;
    const int64_t xcd = bid & 7, local = bid >> 3;
    // Per XCD, groups of 8 row tiles: one column tile after another, each across the
    // group's 8 row tiles (so consecutive workgroups share the column tiles they load).
    const int64_t grp = local / (8 * a.n_tiles_n), rr = local % (8 * a.n_tiles_n);
    const int64_t tile_n = rr / 8;
    const int64_t tile_m = (grp * 8 + rr % 8) * 8 + xcd;
    if (tile_m >= a.n_tiles_m) return;

    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int wm = wave >> 1, wn = wave & 1;
    const int64_t row0 = tile_m * BM;
    const int col0 = (int)tile_n * NB;

    // Started by the first k-step's MFMAs (a zero accumulator operand), not cleared.
    f4 accm[4][TW], accc[4][TW];

    // Stage fill: wave load i (i = 4 j + wave) moves one 1 KB tile (16 rows or columns by
    // 32 k) straight from global memory into LDS, lane l's 16 bytes at byte 16 l.  Row
    // tiles past the chunk's last re-read the last one (their results are masked).
    const int64_t nv = a.n_dev ? *a.n_dev : a.n;   // real rows (loads stay within the n rows)
    const int64_t gmax = (a.n - 1) / 16;          // last row tile of the chunk
    const int64_t tk = a.DP / 32;                 // tiles per row tile
    const uint16_t* src[PW];
#pragma unroll
    for (int j = 0; j < PW; ++j) {
        const int i = 4 * j + wave;
        const int byte = i * 1024;
        if (byte < 2 * A_BYTES) {
            int64_t g = tile_m * (BM / 16) + (byte % A_BYTES) / 1024;
            g = g <= gmax ? g : gmax;
            src[j] = (byte < A_BYTES ? a.Xh : a.Xl) + g * tk * 512 + 8 * lane;
        } else {
            const int bb = byte - 2 * A_BYTES;
            const int64_t g = col0 / 16 + (bb % B_BYTES) / 1024;
            src[j] = (bb < B_BYTES ? a.Wh : a.Wl) + g * tk * 512 + 8 * lane;
        }
    }
    auto fill = [&](char* stage, int k0) {
#pragma unroll
        for (int j = 0; j < PW; ++j)
            load_to_lds16(src[j] + 16 * k0, stage + (4 * j + wave) * 1024);
    };

    // Fragment reads: lane l supplies k = 8 (l >> 4) .. +7 of row / column l & 15, the
    // logical chunk l >> 4 of that tile row.
    const int fr = lane & 15;
    const int foff = fr * 64 + 16 * ((lane >> 4) ^ tile_chunk_swz(fr));
    auto step = [&](const char* stage, auto first) {
        constexpr bool FIRST = decltype(first)::value;
        const f4 z = f4{0.f, 0.f, 0.f, 0.f};
        bf8 ah[4], al[4], bh[TW], bl[TW];
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            const int o = (wm * 64 + 16 * b) * 64 + foff;
            ah[b] = *reinterpret_cast<const bf8*>(stage + o);
            al[b] = *reinterpret_cast<const bf8*>(stage + A_BYTES + o);
        }
#pragma unroll
        for (int t = 0; t < TW; ++t) {
            const int o = (wn * TW + t) * 16 * 64 + foff;
            bh[t] = *reinterpret_cast<const bf8*>(stage + 2 * A_BYTES + o);
            bl[t] = *reinterpret_cast<const bf8*>(stage + 2 * A_BYTES + B_BYTES + o);
        }
#pragma unroll
        for (int t = 0; t < TW; ++t) {
#pragma unroll
            for (int b = 0; b < 4; ++b)
                accm[b][t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[b], bh[t], FIRST ? z : accm[b][t], 0, 0, 0);
#pragma unroll
            for (int b = 0; b < 4; ++b)
                accc[b][t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[b], bl[t], FIRST ? z : accc[b][t], 0, 0, 0);
#pragma unroll
            for (int b = 0; b < 4; ++b)
                accc[b][t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[b], bh[t], accc[b][t], 0, 0, 0);
        }
    };
    const std::false_type later{};

    // Two LDS stages: while one is read by the MFMAs, the next k-step streams into the
    // other.  One barrier per k-step: after it, stage s is complete and every wave has
    // finished reading stage s ^ 1 (its fragments were consumed by the previous step).
    const int nk = a.DP / BK;
    fill(st0, 0);
    wait_lds_loads();
    __syncthreads();
    if (1 < nk) fill(st1, BK);
    step(st0, std::true_type{});
    for (int it = 1; it < nk; it += 2) {  // k-step it from stage 1, it + 1 from stage 0
        wait_lds_loads();
        __syncthreads();
        if (it + 1 < nk) fill(st0, (it + 1) * BK);
        step(st1, later);
        if (it + 1 >= nk) break;
        wait_lds_loads();
        __syncthreads();
        if (it + 2 < nk) fill(st1, (it + 2) * BK);
        step(st0, later);
    }
    const int kin = lane >> 4, cl = lane & 15;
    const uint32_t kmask = (a.K >= 16) ? 0xFFFFu : ((1u << a.K) - 1u);
    const int64_t orow = row0 + wm * 64 + lane;
    const int pick = 4 * kin + (lane & 3), sh = 16 * ((lane & 15) >> 2);
    uint32_t n_ref = 0, n_flip = 0, n_unc = 0;
    const int64_t rw = row0 + wm * 64;  // this wave's first row
    uint32_t rok = 0xFFFFu;             // rows past the batch (last row tile only) take no bits
    if (rw + 64 > nv) {
        rok = 0;
#pragma unroll
        for (int e = 0; e < 16; ++e) rok |= (rw + 16 * (e >> 2) + 4 * kin + (e & 3) < nv) ? (1u << e) : 0u;
    }
    // Row norms of this lane's 16 rows (four consecutive rows per row block): one 16-byte
    // load per block and norm where the wave's rows all exist and the arrays are 16-byte
    // aligned; otherwise one value at a time, rows past n reading row n-1's values (which
    // only matter for rows that store nothing).
    float rA[4][4], rB[4][4], rC[4][4];
    const bool vec_norms = rw + 64 <= a.n && ((reinterpret_cast<uintptr_t>(a.rowA) | reinterpret_cast<uintptr_t>(a.rowB) |
                                               reinterpret_cast<uintptr_t>(a.rowC)) & 15u) == 0;
    if (vec_norms) {
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            const int64_t g = rw + 16 * b + 4 * kin;
            const f4 va = *reinterpret_cast<const f4*>(a.rowA + g), vb = *reinterpret_cast<const f4*>(a.rowB + g),
                     vc = *reinterpret_cast<const f4*>(a.rowC + g);
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                rA[b][r] = va[r];
                rB[b][r] = vb[r];
                rC[b][r] = vc[r];
            }
        }
    } else {
#pragma unroll
        for (int b = 0; b < 4; ++b)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                int64_t g = rw + 16 * b + 4 * kin + r;
                g = g < a.n ? g : a.n - 1;
                rA[b][r] = a.rowA[g];
                rB[b][r] = a.rowB[g];
                rC[b][r] = a.rowC[g];
            }
    }
    float rAm = rA[0][0], rBm = rB[0][0], rCm = rC[0][0];
#pragma unroll
    for (int e = 1; e < 16; ++e) {
        rAm = __builtin_elementwise_maximum(rAm, rA[e >> 2][e & 3]);
        rBm = __builtin_elementwise_maximum(rBm, rB[e >> 2][e & 3]);
        rCm = __builtin_elementwise_maximum(rCm, rC[e >> 2][e & 3]);
    }
    bool fast = true;  // wave-uniform
#pragma unroll
    for (int t = 0; t < TW; ++t) {
        const int table = (col0 >> 4) + wn * TW + t;
        const int cp = col0 + (wn * TW + t) * 16 + cl;
        const float cA = a.wbA[cp], cB = a.wbB[cp], cC = a.wbC[cp], cE = a.wbE[cp];
        f4 p[4];
#pragma unroll
        for (int b = 0; b < 4; ++b) p[b] = accm[b][t] + accc[b][t];
        // Bit e of umask: element e lies inside its bound (NaN is uncertain too).  First one
        // comparison of the smallest |p| against the bound of the lane's largest row factors
        // (every factor is >= 0, so that bound is the largest; minimum and maximum keep a
        // NaN), then, only where that fails somewhere in the wave, element by element.  Once
        // the pre-check has failed, the later tables skip it (data whose bounds are often hit
        // would pay for both).
        const bool chk = a.refine && cA >= 0.f;
        bool exact = !fast;
        if (fast) {
            float amin = fabsf(p[0][0]);
#pragma unroll
            for (int e = 1; e < 16; ++e) amin = __builtin_elementwise_minimum(amin, fabsf(p[e >> 2][e & 3]));
            exact = __any(chk && !(amin > fmaf(rCm, cC, fmaf(rBm, cB, fmaf(rAm, cA, cE)))));
            fast = !exact;
        }
        uint32_t umask = 0;
        if (exact) {
            // (The empty asm keeps the 16 bounds from being computed ahead of the test.)
            float cAv = cA;
            asm volatile("" : "+v"(cAv));
            if (chk) {
#pragma unroll
                for (int e = 0; e < 16; ++e) {
                    float thr = fmaf(rA[e >> 2][e & 3], cAv, cE);
                    thr = fmaf(rB[e >> 2][e & 3], cB, thr);
                    thr = fmaf(rC[e >> 2][e & 3], cC, thr);
                    umask |= !(fabsf(p[e >> 2][e & 3]) > thr) ? (1u << e) : 0u;
                }
                umask &= rok;
            }
        }
        if (a.refine == 2) {
            n_unc += __popc(umask);  // count only: the raw signs stand
            umask = 0;
        }
        if (__any(umask != 0)) {
            const uint32_t mine = __popc(umask);
            uint32_t incl = mine;
#pragma unroll
            for (int off = 1; off < 64; off <<= 1) {
                const uint32_t v = __shfl_up(incl, off, 64);
                if (lane >= off) incl += v;
            }
            const uint32_t total = __shfl(incl, 63, 64);
            u64 base = 0;
            if (lane == 0) base = atomicAdd(a.list_count, (u64)total);
            base = __shfl(base, 0, 64);
            u64 slot = base + (incl - mine);
            for (int e = 0; e < 16; ++e) {
                if (!((umask >> e) & 1u)) continue;
                const int64_t grow = row0 + wm * 64 + 16 * (e >> 2) + 4 * kin + (e & 3);
                const float pv = p[e >> 2][e & 3];
                if (slot < a.list_cap) {
                    a.list[slot] = (u64)(uint32_t)grow | ((u64)cp << 32) | ((pv > 0.f) ? (1ull << 63) : 0ull);
                } else {
                    const float* xr = a.X + grow * (int64_t)a.d;
                    const float* wr = a.Wt + (int64_t)cp * a.DP;
                    double sacc = 0.0;
                    for (int u = 0; u < a.d; ++u) sacc += (double)xr[u] * (double)wr[u];
                    mark_refined(a, grow, cp);
                    n_ref += 1u;
                    n_flip += ((sacc > 0.0) != (pv > 0.f)) ? 1u : 0u;
                    p[e >> 2][e & 3] = sacc > 0.0 ? 1.f : -1.f;
                }
                ++slot;
            }
        }
        uint32_t f[16];
#pragma unroll
        for (int e = 0; e < 16; ++e) {
            f[e] = (uint32_t)(__ballot(p[e >> 2][e & 3] > 0.f) >> sh);
            // Shift each ballot as it is taken: selecting the unshifted scalar pairs first
            // would cost two vector selects (and copies) per pair.
            asm("" : "+v"(f[e]));
        }
        const uint32_t code = pick_code(f, pick);
        if (table < a.L && orow < nv) a.codes[(int64_t)table * a.ldc + orow] = (uint16_t)(code & kmask);
    }
    if (__any(n_ref != 0 || n_unc != 0)) {
        const uint32_t r = wave_sum_u32(n_ref), f = wave_sum_u32(n_flip), uc = wave_sum_u32(n_unc);
        if (lane == 0) {
            if (r) atomicAdd(&a.counters[0], (u64)r);
            if (f) atomicAdd(&a.counters[1], (u64)f);
            if (uc) atomicAdd(&a.counters[2], (u64)uc);
        }
    }
}

template <int TW>
hipError_t launch_tw(const HashArgs& a, hipStream_t s) {
    const int64_t groups = (a.n_tiles_m + 63) / 64;
    const int64_t blocks = groups * 64 * a.n_tiles_n;
    hipLaunchKernelGGL((hash_bf16_kernel<TW>), dim3((unsigned)blocks), dim3(256), 0, s, a);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_convert_bf16(const float* X, int64_t n, int d, int DP, bool vec, uint16_t* Xh, uint16_t* Xl,
                               float* rowA, float* rowB, float* rowC, float norm_up, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    const int64_t n16 = (n + 15) / 16 * 16;
    const int lpr = DP >= 256 ? 64 : DP >= 128 ? 32 : DP >= 64 ? 16 : 8;  // DP is a multiple of 32
    const int64_t rows_per_block = 4 * (64 / lpr);
    const int64_t blocks = (n16 + rows_per_block - 1) / rows_per_block;
#define ACE_CONVERT(V, P)                                                                                     \
    hipLaunchKernelGGL((convert_bf16_kernel<V, P>), dim3((unsigned)blocks), dim3(256), 0, s, X, n, n16, d, DP, \
                       Xh, Xl, rowA, rowB, rowC, norm_up)
    switch (lpr) {
        case 64: if (vec) ACE_CONVERT(true, 64); else ACE_CONVERT(false, 64); break;
        case 32: if (vec) ACE_CONVERT(true, 32); else ACE_CONVERT(false, 32); break;
        case 16: if (vec) ACE_CONVERT(true, 16); else ACE_CONVERT(false, 16); break;
        default: if (vec) ACE_CONVERT(true, 8); else ACE_CONVERT(false, 8); break;
    }
#undef ACE_CONVERT
    return hipGetLastError();
}

hipError_t launch_hash_bf16(const HashArgs& a, int TW, hipStream_t s) {
    switch (TW) {
        case 1: return launch_tw<1>(a, s);
        case 2: return launch_tw<2>(a, s);
        case 4: return launch_tw<4>(a, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace ace
