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
// bounded by Cauchy-Schwarz.  Accumulation error: an MFMA aligns the products of a
// step to the largest magnitude among them and the accumulator and drops bits below
// that (measured on gfx950), so each instruction can lose up to (terms + 2) units of
// 2^-23 relative to |accumulator| + sum|products|; over a chain of I instructions
// this is at most (34 I) u sum|products| with u = 2^-23 (32 products per
// instruction).  Hence, with A = ||x_h||, B = ||x_l||, C = ||rho_x||:
//     |p - p~| <= A cA_c + B cB_c + C cC_c + eps_c
//     cA = ||rho_w|| + (34 I u) ||w_h|| + (68 I u) ||w_l|| + 2u (||w_h|| + ||w_l||)
//     cB = ||w_l|| + ||rho_w|| + (68 I u) ||w_h|| + 2u ||w_h||
//     cC = ||w||
// (I = padded d / 32; eps_c covers flushed subnormal products), all rounded up by
// the host.  Outside the bound the sign of p~ is the sign of p; inside it the
// projection is queued for the FP64 pass, exactly as in the FP32 kernel.
//
// Tiling: 256 threads = 4 waves as 2 (rows) x 2 (columns); workgroup tile 128 rows
// x 2*TW tables (TW <= 4); per wave 64 rows x TW tables, 2 x 4 x TW accumulators of
// 16x16.  The register budget (256 per lane) keeps two waves per SIMD.
// The FP32 X tile is converted to hi/lo in registers on its way to LDS, together
// with the three row norms (FP32 sums of squares, rounded up at the end).
#include "ace_internal.h"

namespace ace {

namespace {

constexpr int BM = 128;
constexpr int BK = 32;
constexpr int LDSB = BK + 8;  // padded LDS row stride in bf16 elements (80 bytes)

typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef short s8v __attribute__((ext_vector_type(8)));
typedef short s4v __attribute__((ext_vector_type(4)));

__device__ inline uint32_t select_code(u64 m0, u64 m1, u64 m2, u64 m3, int lane) {
    const int r = lane & 3, g = (lane & 15) >> 2;
    u64 m = r == 0 ? m0 : r == 1 ? m1 : r == 2 ? m2 : m3;
    return (uint32_t)(m >> (16 * g)) & 0xFFFFu;
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

template <int TW, bool VEC>
__global__ __launch_bounds__(256) void hash_bf16_kernel(const HashArgs a) {
    constexpr int NB = 32 * TW;
    __shared__ uint16_t Xh[BM * LDSB], Xl[BM * LDSB];
    __shared__ uint16_t Wh[NB * LDSB], Wl[NB * LDSB];
    __shared__ __attribute__((aligned(16))) float rowA[BM], rowB[BM], rowC[BM];

    const int64_t bid = blockIdx.x;
    const int64_t xcd = bid & 7, local = bid >> 3;
    const int64_t tile_n = local % a.n_tiles_n;
    const int64_t tile_m = (local / a.n_tiles_n) * 8 + xcd;
    if (tile_m >= a.n_tiles_m) return;

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave >> 1, wn = wave & 1;
    const int64_t row0 = tile_m * BM;
    const int col0 = (int)tile_n * NB;

    f4 accm[4][TW], accc[4][TW];
#pragma unroll
    for (int b = 0; b < 4; ++b)
#pragma unroll
        for (int t = 0; t < TW; ++t) {
            accm[b][t] = f4{0.f, 0.f, 0.f, 0.f};
            accc[b][t] = f4{0.f, 0.f, 0.f, 0.f};
        }

    const int lr = tid >> 1, lk = (tid & 1) * 16;
    const int64_t grow_ld = row0 + lr;
    const bool row_ok = grow_ld < a.n;
    const float* xrow = a.X + (row_ok ? grow_ld : 0) * (int64_t)a.d;
    float sA = 0.f, sB = 0.f, sC = 0.f;

    // The next chunk's X values and W quads are fetched into registers while the
    // current chunk's MFMAs run.
    float xv[16];
    s4v whv[TW], wlv[TW];
    auto gload = [&](int k0) {
        if (VEC) {
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int k = k0 + lk + 4 * q;
                f4 t = f4{0.f, 0.f, 0.f, 0.f};
                if (row_ok && k < a.d) t = *reinterpret_cast<const f4*>(xrow + k);
                xv[4 * q] = t[0];
                xv[4 * q + 1] = t[1];
                xv[4 * q + 2] = t[2];
                xv[4 * q + 3] = t[3];
            }
        } else {
#pragma unroll
            for (int e = 0; e < 16; ++e) {
                const int k = k0 + lk + e;
                xv[e] = (row_ok && k < a.d) ? xrow[k] : 0.f;
            }
        }
#pragma unroll
        for (int s = 0; s < TW; ++s) {
            const int q = tid + 256 * s;
            const int64_t gi = (int64_t)(col0 + (q >> 3)) * a.DP + k0 + (q & 7) * 4;
            whv[s] = *reinterpret_cast<const s4v*>(a.Wh + gi);
            wlv[s] = *reinterpret_cast<const s4v*>(a.Wl + gi);
        }
    };

    gload(0);
    for (int k0 = 0; k0 < a.d; k0 += BK) {
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            s8v ph, pl;
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const float x = xv[8 * h + e];
                const uint16_t hb = bf16_bits(x);
                const float hv = bf16_val(hb);
                const float r1 = x - hv;  // exact
                const uint16_t lb = bf16_bits(r1);
                const float lv = bf16_val(lb);
                const float r2 = r1 - lv;  // exact
                sA = fmaf(hv, hv, sA);
                sB = fmaf(lv, lv, sB);
                sC = fmaf(r2, r2, sC);
                ph[e] = (short)hb;
                pl[e] = (short)lb;
            }
            *reinterpret_cast<s8v*>(Xh + lr * LDSB + lk + 8 * h) = ph;
            *reinterpret_cast<s8v*>(Xl + lr * LDSB + lk + 8 * h) = pl;
        }
#pragma unroll
        for (int s = 0; s < TW; ++s) {
            const int q = tid + 256 * s;
            const int off = (q >> 3) * LDSB + (q & 7) * 4;
            *reinterpret_cast<s4v*>(Wh + off) = whv[s];
            *reinterpret_cast<s4v*>(Wl + off) = wlv[s];
        }
        __syncthreads();
        if (k0 + BK < a.d) gload(k0 + BK);
        // Lane l supplies k = 8*(l>>4) .. +7 of row/column (l & 15) for one 16x16x32 step.
        bf8 ah[4], al[4];
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            const int off = (wm * 64 + 16 * b + (lane & 15)) * LDSB + 8 * (lane >> 4);
            ah[b] = *reinterpret_cast<const bf8*>(Xh + off);
            al[b] = *reinterpret_cast<const bf8*>(Xl + off);
        }
#pragma unroll
        for (int t = 0; t < TW; ++t) {
            const int off = ((wn * TW + t) * 16 + (lane & 15)) * LDSB + 8 * (lane >> 4);
            const bf8 bh = *reinterpret_cast<const bf8*>(Wh + off);
            const bf8 bl = *reinterpret_cast<const bf8*>(Wl + off);
#pragma unroll
            for (int b = 0; b < 4; ++b) {
                accm[b][t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[b], bh, accm[b][t], 0, 0, 0);
                accc[b][t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[b], bl, accc[b][t], 0, 0, 0);
                accc[b][t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[b], bh, accc[b][t], 0, 0, 0);
            }
        }
        __syncthreads();
    }

    // Row norms: the pair of threads of each row combine; FP32 sums of squares of d
    // terms are rounded up by gamma_{d+2}(2^-24) and the square root by 2^-20.
    sA += __shfl_xor(sA, 1, 64);
    sB += __shfl_xor(sB, 1, 64);
    sC += __shfl_xor(sC, 1, 64);
    if ((tid & 1) == 0) {
        rowA[lr] = sqrtf(sA * a.norm_up) * (1.f + 0x1p-20f);
        rowB[lr] = sqrtf(sB * a.norm_up) * (1.f + 0x1p-20f);
        rowC[lr] = sqrtf(sC * a.norm_up) * (1.f + 0x1p-20f);
    }
    __syncthreads();

    const int kin = lane >> 4, cl = lane & 15;
    const uint32_t kmask = (a.K >= 16) ? 0xFFFFu : ((1u << a.K) - 1u);
    const int64_t orow = row0 + wm * 64 + lane;
    uint32_t n_ref = 0, n_flip = 0;
    uint32_t rok = 0;
#pragma unroll
    for (int e = 0; e < 16; ++e)
        rok |= (row0 + wm * 64 + 16 * (e >> 2) + 4 * kin + (e & 3) < a.n) ? (1u << e) : 0u;
    f4 rA[4], rB[4], rC[4];
#pragma unroll
    for (int b = 0; b < 4; ++b) {
        const int lrow = wm * 64 + 16 * b + 4 * kin;
        rA[b] = *reinterpret_cast<const f4*>(rowA + lrow);
        rB[b] = *reinterpret_cast<const f4*>(rowB + lrow);
        rC[b] = *reinterpret_cast<const f4*>(rowC + lrow);
    }
#pragma unroll
    for (int t = 0; t < TW; ++t) {
        const int table = (col0 >> 4) + wn * TW + t;
        const int cp = col0 + (wn * TW + t) * 16 + cl;
        const float cA = a.wbA[cp], cB = a.wbB[cp], cC = a.wbC[cp], cE = a.wbE[cp];
        f4 p[4];
#pragma unroll
        for (int b = 0; b < 4; ++b) p[b] = accm[b][t] + accc[b][t];
        uint32_t umask = 0;
        if (a.refine && cA >= 0.f) {
#pragma unroll
            for (int e = 0; e < 16; ++e) {
                float thr = fmaf(rA[e >> 2][e & 3], cA, cE);
                thr = fmaf(rB[e >> 2][e & 3], cB, thr);
                thr = fmaf(rC[e >> 2][e & 3], cC, thr);
                umask |= !(fabsf(p[e >> 2][e & 3]) > thr) ? (1u << e) : 0u;
            }
            umask &= rok;
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
                    n_ref += 1u;
                    n_flip += ((sacc > 0.0) != (pv > 0.f)) ? 1u : 0u;
                    p[e >> 2][e & 3] = sacc > 0.0 ? 1.f : -1.f;
                }
                ++slot;
            }
        }
        uint32_t code = 0;
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            const uint32_t cb = select_code(__ballot(p[b][0] > 0.f), __ballot(p[b][1] > 0.f),
                                            __ballot(p[b][2] > 0.f), __ballot(p[b][3] > 0.f), lane);
            code = (kin == b) ? cb : code;
        }
        if (table < a.L && orow < a.n) a.codes[(int64_t)table * a.ldc + orow] = (uint16_t)(code & kmask);
    }
    if (__any(n_ref != 0)) {
        const uint32_t r = wave_sum_u32(n_ref), f = wave_sum_u32(n_flip);
        if (lane == 0) {
            atomicAdd(&a.counters[0], (u64)r);
            if (f) atomicAdd(&a.counters[1], (u64)f);
        }
    }
}

template <int TW>
hipError_t launch_tw(const HashArgs& a, bool vec, hipStream_t s) {
    const int64_t groups = (a.n_tiles_m + 7) / 8;
    const int64_t blocks = groups * 8 * a.n_tiles_n;
    if (vec)
        hipLaunchKernelGGL((hash_bf16_kernel<TW, true>), dim3((unsigned)blocks), dim3(256), 0, s, a);
    else
        hipLaunchKernelGGL((hash_bf16_kernel<TW, false>), dim3((unsigned)blocks), dim3(256), 0, s, a);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_hash_bf16(const HashArgs& a, int TW, bool vec, hipStream_t s) {
    switch (TW) {
        case 1: return launch_tw<1>(a, vec, s);
        case 2: return launch_tw<2>(a, vec, s);
        case 4: return launch_tw<4>(a, vec, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace ace
