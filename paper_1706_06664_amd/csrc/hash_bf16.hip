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
// 16x16.  The register budget (256 per lane) keeps two waves per SIMD.  X is split
// into hi/lo once per chunk by convert_bf16_kernel (which also writes the three row
// norms); the projection kernel then streams pre-split bf16 tiles.
#include "ace_internal.h"

namespace ace {

namespace {

constexpr int BM = 128;
constexpr int BK = 32;
constexpr int LDSB = BK + 16;  // padded LDS row stride in bf16 elements (96 bytes: the 16-byte fragment reads of 16 rows hit distinct banks)

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

// Convert + row norms: X (FP32 [n][d]) -> Xh, Xl (bf16 bits [n][DP], zero-padded to
// DP) and the row norms A = ||x_h||, B = ||x_l||, C = ||rho_x|| (FP32 sums of squares
// rounded up by norm_up, square roots by 2^-20).  One wave per row; lane l takes the 4
// consecutive k at 4l + 256i (a wave instruction reads 1 KB contiguous) and writes 8
// bytes of hi and 8 of lo.
template <bool VEC>
__global__ __launch_bounds__(256) void convert_bf16_kernel(const float* __restrict__ X, int64_t n, int d, int DP,
                                                           uint16_t* __restrict__ Xh, uint16_t* __restrict__ Xl,
                                                           float* __restrict__ rowA, float* __restrict__ rowB,
                                                           float* __restrict__ rowC, float norm_up) {
    const int lane = threadIdx.x & 63;
    const int64_t row = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (row >= n) return;
    const float* xr = X + row * (int64_t)d;
    float sA = 0.f, sB = 0.f, sC = 0.f;
    for (int k0 = 4 * lane; k0 < DP; k0 += 256) {
        f4 v;
        if (VEC && k0 + 4 <= d) {
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
        // streamed in and out: the projection kernel reads the split rows back much later
        __builtin_nontemporal_store(ph, reinterpret_cast<s4v*>(Xh + row * (int64_t)DP + k0));
        __builtin_nontemporal_store(pl, reinterpret_cast<s4v*>(Xl + row * (int64_t)DP + k0));
    }
    for (int off = 32; off > 0; off >>= 1) {
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

template <int TW>
__global__ __launch_bounds__(256, 2) void hash_bf16_kernel(const HashArgs a) {
    constexpr int NB = 32 * TW;
    __shared__ uint16_t Xh[BM * LDSB], Xl[BM * LDSB];
    __shared__ uint16_t Wh[NB * LDSB], Wl[NB * LDSB];

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

    // A-tile role: thread -> row lr, 16 consecutive k at lk, hi and lo (two 16-byte
    // loads each).  The next chunk is fetched into registers while the current chunk's
    // MFMAs run.
    const int lr = tid >> 1, lk = (tid & 1) * 16;
    const int64_t grow_ld = row0 + lr;
    const int64_t nv = a.n_dev ? *a.n_dev : a.n;   // real rows (loads stay within the n rows)
    const bool row_ok = grow_ld < a.n;
    const uint16_t* xh = a.Xh + (row_ok ? grow_ld : 0) * (int64_t)a.DP + lk;
    const uint16_t* xl = a.Xl + (row_ok ? grow_ld : 0) * (int64_t)a.DP + lk;
    s8v xhv[2], xlv[2];
    s4v whv[TW], wlv[TW];
    auto gload = [&](int k0) {
        // rows past n read row 0 of the chunk (their results are masked)
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            xhv[h] = *reinterpret_cast<const s8v*>(xh + k0 + 8 * h);
            xlv[h] = *reinterpret_cast<const s8v*>(xl + k0 + 8 * h);
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
    for (int k0 = 0; k0 < a.DP; k0 += BK) {
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            *reinterpret_cast<s8v*>(Xh + lr * LDSB + lk + 8 * h) = xhv[h];
            *reinterpret_cast<s8v*>(Xl + lr * LDSB + lk + 8 * h) = xlv[h];
        }
#pragma unroll
        for (int s = 0; s < TW; ++s) {
            const int q = tid + 256 * s;
            const int off = (q >> 3) * LDSB + (q & 7) * 4;
            *reinterpret_cast<s4v*>(Wh + off) = whv[s];
            *reinterpret_cast<s4v*>(Wl + off) = wlv[s];
        }
        __syncthreads();
        if (k0 + BK < a.DP) gload(k0 + BK);
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

    const int kin = lane >> 4, cl = lane & 15;
    const uint32_t kmask = (a.K >= 16) ? 0xFFFFu : ((1u << a.K) - 1u);
    const int64_t orow = row0 + wm * 64 + lane;
    uint32_t n_ref = 0, n_flip = 0, n_unc = 0;
    uint32_t rok = 0;
#pragma unroll
    for (int e = 0; e < 16; ++e)
        rok |= (row0 + wm * 64 + 16 * (e >> 2) + 4 * kin + (e & 3) < nv) ? (1u << e) : 0u;
    // Row norms of this lane's 16 rows (four consecutive rows per row block); rows past
    // n read row n-1's values, which only matter for rows that store nothing.
    float rA[4][4], rB[4][4], rC[4][4];
#pragma unroll
    for (int b = 0; b < 4; ++b)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            int64_t g = row0 + wm * 64 + 16 * b + 4 * kin + r;
            g = g < a.n ? g : a.n - 1;
            rA[b][r] = a.rowA[g];
            rB[b][r] = a.rowB[g];
            rC[b][r] = a.rowC[g];
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
        uint32_t code = 0;
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            const uint32_t cb = select_code(__ballot(p[b][0] > 0.f), __ballot(p[b][1] > 0.f),
                                            __ballot(p[b][2] > 0.f), __ballot(p[b][3] > 0.f), lane);
            code = (kin == b) ? cb : code;
        }
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
    const int64_t groups = (a.n_tiles_m + 7) / 8;
    const int64_t blocks = groups * 8 * a.n_tiles_n;
    hipLaunchKernelGGL((hash_bf16_kernel<TW>), dim3((unsigned)blocks), dim3(256), 0, s, a);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_convert_bf16(const float* X, int64_t n, int d, int DP, bool vec, uint16_t* Xh, uint16_t* Xl,
                               float* rowA, float* rowB, float* rowC, float norm_up, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    const int64_t blocks = (n + 3) / 4;
    if (vec)
        hipLaunchKernelGGL(convert_bf16_kernel<true>, dim3((unsigned)blocks), dim3(256), 0, s, X, n, d, DP, Xh, Xl,
                           rowA, rowB, rowC, norm_up);
    else
        hipLaunchKernelGGL(convert_bf16_kernel<false>, dim3((unsigned)blocks), dim3(256), 0, s, X, n, d, DP, Xh, Xl,
                           rowA, rowB, rowC, norm_up);
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
