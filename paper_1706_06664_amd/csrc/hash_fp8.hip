// SRP hashing on FP8 (OCP e4m3) MFMA with power-of-two row and column scales
// (Sec. 2.1 signed random projections, Sec. 3.2 K-bit codes),
// v_mfma_scale_f32_16x16x128_f8f6f4 with unit block scales, FP32 accumulate.
//
// Each row is scaled by s_i = 2^ceil(log2(max|x_i| / 448)) and each W column by s_c
// likewise, so every scaled value fits e4m3 (max 448) and scaling is exact.  The
// kernel computes p^ = sum_t x^_t w^_t in scaled units; positive scales do not change
// the sign, so p^ decides the bit.  With x/s = x^ + dx and w/s_c = w^ + dw (both
// remainders exact in FP32):
//     |p/(s_i s_c) - p^| <= ||x^|| ||dw|| + ||dx|| ||w^|| + ||dx|| ||dw|| + acc
// where acc bounds the accumulation.  On gfx950 the unit aligns the 8 products of a
// k-group to the largest and keeps about 13 bits below it (measured), then adds group
// sums to the FP32 accumulator with round-to-nearest, so
//     acc <= (2^-9 + 8 I 2^-24) sum |x^ w^|,  I = DP / 128 instructions
// (twice the measured in-group loss).  The bound is A cA + B cB + eps with
// A = ||x^||, B = ||dx|| and cA = ||dw|| + (2^-9 + 8 I 2^-24) ||w^||,
// cB = ||w^|| + ||dw||, rounded up by the host.  Projections inside it are queued for
// the FP64 pass (refine = 1) or only counted (refine = 2).
//
// Tiling as in the BF16 kernel: 256 threads = 2 x 2 waves, 128 rows x 2*TW tables per
// workgroup, k-steps of 128 (one MFMA).  Rows and columns are stored in 16 x 128 tiles
// (fp8_tiled_index); each k-step moves whole tiles from global memory straight into one
// of two LDS stages while the MFMAs read the other.  Lane l supplies the 16 k of chunk
// l / 16 from both 64-byte halves of its row or column (the same k for both operands).
#include <type_traits>

#include "ace_internal.h"

namespace ace {

namespace {

constexpr int BM = 128;
constexpr int BKB = 128;            // k per step (bytes per row of a tile)

typedef float f4 __attribute__((ext_vector_type(4)));
typedef int i8v __attribute__((ext_vector_type(8)));
typedef int i4v __attribute__((ext_vector_type(4)));

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

// OCP e4m3 (bias 7, max 448, subnormals q * 2^-9) with round-to-nearest-even, for
// |v| <= 448.  Returns the code and the value it encodes.
__device__ inline uint32_t e4m3_encode(float v, float& q) {
    const uint32_t s = (__float_as_uint(v) >> 24) & 0x80u;
    const float a = fabsf(v);
    if (a < 0x1p-6f) {
        const float m = rintf(a * 512.f);  // 0..8; 8 is the smallest normal, same code
        q = copysignf(m * 0x1p-9f, v);
        return s | (uint32_t)m;
    }
    uint32_t u = __float_as_uint(a);
    u += 0x7FFFFu + ((u >> 20) & 1u);      // round the mantissa to 3 bits
    u &= 0xFFF00000u;
    q = copysignf(__uint_as_float(u), v);
    const uint32_t E = ((u >> 23) & 0xFFu) - 127u + 7u;
    const uint32_t M = (u >> 20) & 7u;
    return s | (E << 3) | M;
}

// Convert + row norms: one wave per row.  Lane l takes the 4 consecutive k at
// 4l + 256i (one 16-byte load; a wave instruction reads 1 KB contiguous).  Rows of up
// to RCACHE*256 values stay in registers between the max pass and the encode pass.
constexpr int RCACHE = 16;

__device__ inline f4 load4(const float* xr, int k, int d, bool vec) {
    if (vec && k + 4 <= d) return *reinterpret_cast<const f4*>(xr + k);
    f4 v;
#pragma unroll
    for (int e = 0; e < 4; ++e) v[e] = (k + e < d) ? xr[k + e] : 0.f;
    return v;
}

template <bool VEC>
__global__ __launch_bounds__(256) void convert_fp8_kernel(const float* __restrict__ X, int64_t n, int64_t n16, int d, int DP,
                                                          uint8_t* __restrict__ Xq, float* __restrict__ rowA,
                                                          float* __restrict__ rowB, float norm_up) {
    const int lane = threadIdx.x & 63;
    const int64_t row = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (row >= n16) return;
    if (row >= n) {  // rows n .. n16-1 fill the last 16-row tile with zeros
        for (int k = 4 * lane; k < DP; k += 256) *reinterpret_cast<uint32_t*>(Xq + fp8_tiled_index(row, k, DP)) = 0u;
        return;
    }
    const float* xr = X + row * (int64_t)d;
    f4 cache[RCACHE];
    float mx = 0.f;
#pragma unroll
    for (int i = 0; i < RCACHE; ++i) {
        cache[i] = f4{0.f, 0.f, 0.f, 0.f};
        if (i * 256 < DP) {
            cache[i] = load4(xr, 4 * lane + 256 * i, d, VEC);
            mx = fmaxf(mx, fmaxf(fmaxf(fabsf(cache[i][0]), fabsf(cache[i][1])),
                                 fmaxf(fabsf(cache[i][2]), fabsf(cache[i][3]))));
        }
    }
    for (int k = 4 * lane + 256 * RCACHE; k < DP; k += 256) {
        const f4 v = load4(xr, k, d, VEC);
        mx = fmaxf(mx, fmaxf(fmaxf(fabsf(v[0]), fabsf(v[1])), fmaxf(fabsf(v[2]), fabsf(v[3]))));
    }
    for (int off = 32; off > 0; off >>= 1) mx = fmaxf(mx, __shfl_xor(mx, off, 64));
    // scale exponent: smallest e with max|x| * 2^-e <= 448; multiplying by 2^-e is exact
    int e = 0;
    if (mx > 0.f) {
        e = ilogbf(mx / 448.f);
        while (ldexpf(mx, -e) > 448.f) ++e;
    }
    // The scaling is one exact ldexp per value: 2^-e itself overflows FP32 for rows whose
    // largest value is below about 2^-119.
    float sA = 0.f, sB = 0.f;
    auto encode = [&](f4 v, int k) {
        uint32_t word = 0;
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            const float x = ldexpf(v[b], -e);
            float qv;
            const uint32_t code = e4m3_encode(x, qv) & 0xFFu;
            const float dx = x - qv;  // exact
            sA = fmaf(qv, qv, sA);
            sB = fmaf(dx, dx, sB);
            word |= code << (8 * b);
        }
        // streamed out: the projection kernel reads the rows back much later
        __builtin_nontemporal_store(word, reinterpret_cast<uint32_t*>(Xq + fp8_tiled_index(row, k, DP)));
    };
#pragma unroll
    for (int i = 0; i < RCACHE; ++i)
        if (4 * lane + 256 * i < DP) encode(cache[i], 4 * lane + 256 * i);
    for (int k = 4 * lane + 256 * RCACHE; k < DP; k += 256) encode(load4(xr, k, d, VEC), k);
    for (int off = 32; off > 0; off >>= 1) {
        sA += __shfl_xor(sA, off, 64);
        sB += __shfl_xor(sB, off, 64);
    }
    if (lane == 0) {
        rowA[row] = sqrtf(sA * norm_up) * (1.f + 0x1p-20f);
        rowB[row] = sqrtf(sB * norm_up) * (1.f + 0x1p-20f);
    }
}

// One wave-wide 16-byte-per-lane load from global memory straight into LDS: lane l's
// 16 bytes land at lds + 16 l (lds is the same for every lane).
__device__ inline void load_to_lds16(const uint8_t* g, uint8_t* lds) {
    __builtin_amdgcn_global_load_lds(g, (__attribute__((address_space(3))) void*)lds, 16, 0, 0);
}

// Wait until this wave's loads into LDS have landed.
__device__ inline void wait_lds_loads() { asm volatile("s_waitcnt vmcnt(0)" ::: "memory"); }

template <int TW>
__global__ __launch_bounds__(256, 2) void hash_fp8_kernel(const HashArgs a) {
    constexpr int NB = 32 * TW;
    constexpr int A_BYTES = BM * BKB;                  // rows of one k-step (16 KB)
    constexpr int B_BYTES = NB * BKB;                  // columns of one k-step
    constexpr int STAGE = A_BYTES + B_BYTES;
    constexpr int NI = STAGE / 1024;                   // 1 KB wave loads per stage (16 + 4 TW)
    constexpr int PW = NI / 4;                         // per wave
    static_assert(NI % 4 == 0, "stage loads split evenly over the four waves");
    __shared__ __attribute__((aligned(1024))) uint8_t st0[STAGE];
    __shared__ __attribute__((aligned(1024))) uint8_t st1[STAGE];

    const int64_t bid = blockIdx.x;
    const int64_t xcd = bid & 7, local = bid >> 3;
    const int64_t tile_n = local % a.n_tiles_n;
    const int64_t tile_m = (local / a.n_tiles_n) * 8 + xcd;
    if (tile_m >= a.n_tiles_m) return;

    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int wm = wave >> 1, wn = wave & 1;
    const int64_t row0 = tile_m * BM;
    const int col0 = (int)tile_n * NB;

    f4 acc[4][TW];  // started by the first k-step's products (a zero accumulator operand)

    // Stage fill: wave load i (i = 4 j + wave) moves one 1 KB sub-tile (16 rows or columns,
    // one 64-byte half of the k-step) straight into LDS, lane l's 16 bytes at byte 16 l.
    // Row tiles past the chunk's last re-read the last one (their results are masked).
    const int64_t nv = a.n_dev ? *a.n_dev : a.n;   // real rows (loads stay within the n rows)
    const int64_t gmax = (a.n - 1) / 16;          // last row tile of the chunk
    const int64_t tk = a.DP / BKB;                // tiles per row tile
    const uint8_t* src[PW];
#pragma unroll
    for (int j = 0; j < PW; ++j) {
        const int i = 4 * j + wave;
        if (i < A_BYTES / 1024) {
            int64_t g = tile_m * (BM / 16) + i / 2;
            g = g <= gmax ? g : gmax;
            src[j] = a.Xq + g * tk * 2048 + (i & 1) * 1024 + 16 * lane;
        } else {
            const int ib = i - A_BYTES / 1024;
            const int64_t g = col0 / 16 + ib / 2;
            src[j] = a.Wq + g * tk * 2048 + (ib & 1) * 1024 + 16 * lane;
        }
    }
    auto fill = [&](uint8_t* stage, int k0) {
#pragma unroll
        for (int j = 0; j < PW; ++j) load_to_lds16(src[j] + 16 * k0, stage + (4 * j + wave) * 1024);
    };

    // Fragment reads: lane l takes chunk l / 16 of row / column l & 15 from both halves.
    const int fr = lane & 15;
    const int foff = fr * 64 + 16 * ((lane >> 4) ^ tile_chunk_swz(fr));
    auto frag = [&](const uint8_t* p) {
        const i4v lo = *reinterpret_cast<const i4v*>(p), hi = *reinterpret_cast<const i4v*>(p + 1024);
        return i8v{lo[0], lo[1], lo[2], lo[3], hi[0], hi[1], hi[2], hi[3]};
    };
    auto step = [&](const uint8_t* stage, auto first) {
        constexpr bool FIRST = decltype(first)::value;
        const f4 z = f4{0.f, 0.f, 0.f, 0.f};
        i8v af[4];
#pragma unroll
        for (int b = 0; b < 4; ++b) af[b] = frag(stage + (wm * 4 + b) * 2048 + foff);
#pragma unroll
        for (int t = 0; t < TW; ++t) {
            const i8v bf = frag(stage + A_BYTES + (wn * TW + t) * 2048 + foff);
#pragma unroll
            for (int b = 0; b < 4; ++b)
                acc[b][t] = __builtin_amdgcn_mfma_scale_f32_16x16x128_f8f6f4(af[b], bf, FIRST ? z : acc[b][t], 0, 0,
                                                                             0, 127, 0, 127);
        }
    };

    // Two LDS stages: while one is read by the MFMAs, the next k-step streams into the
    // other.  One barrier per k-step: after it, stage s is complete and every wave has
    // finished reading stage s ^ 1 (its fragments were consumed by the previous step).
    const int nk = a.DP / BKB;
    const std::false_type later{};
    fill(st0, 0);
    wait_lds_loads();
    __syncthreads();
    if (1 < nk) fill(st1, BKB);
    step(st0, std::true_type{});
    for (int it = 1; it < nk; it += 2) {  // k-step it from stage 1, it + 1 from stage 0
        wait_lds_loads();
        __syncthreads();
        if (it + 1 < nk) fill(st0, (it + 1) * BKB);
        step(st1, later);
        if (it + 1 >= nk) break;
        wait_lds_loads();
        __syncthreads();
        if (it + 2 < nk) fill(st1, (it + 2) * BKB);
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
    // Row factors of this lane's 16 rows (four consecutive rows per row block): one 16-byte
    // load per block and factor where the wave's rows all exist and the arrays are 16-byte
    // aligned; otherwise one value at a time, rows past n reading row n-1's values (which
    // only matter for rows that store nothing).
    float rA[16], rB[16];
    const bool vec_norms =
        rw + 64 <= a.n && ((reinterpret_cast<uintptr_t>(a.rowA) | reinterpret_cast<uintptr_t>(a.rowB)) & 15u) == 0;
    if (vec_norms) {
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            const int64_t g = rw + 16 * b + 4 * kin;
            const f4 va = *reinterpret_cast<const f4*>(a.rowA + g), vb = *reinterpret_cast<const f4*>(a.rowB + g);
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                rA[4 * b + r] = va[r];
                rB[4 * b + r] = vb[r];
            }
        }
    } else {
#pragma unroll
        for (int e = 0; e < 16; ++e) {
            int64_t g = rw + 16 * (e >> 2) + 4 * kin + (e & 3);
            g = g < a.n ? g : a.n - 1;
            rA[e] = a.rowA[g];
            rB[e] = a.rowB[g];
        }
    }
    float rAm = rA[0], rBm = rB[0];
#pragma unroll
    for (int e = 1; e < 16; ++e) {
        rAm = __builtin_elementwise_maximum(rAm, rA[e]);
        rBm = __builtin_elementwise_maximum(rBm, rB[e]);
    }
    bool fast = true;  // wave-uniform
#pragma unroll
    for (int t = 0; t < TW; ++t) {
        const int table = (col0 >> 4) + wn * TW + t;
        const int cp = col0 + (wn * TW + t) * 16 + cl;
        const float cA = a.wbA[cp], cB = a.wbB[cp], cE = a.wbE[cp];
        // Bit e of umask: element e lies inside its bound (NaN is uncertain too).  First one
        // comparison of the smallest |p| against the bound of the lane's largest row factors
        // (every factor is >= 0, so that bound is the largest; minimum and maximum keep a
        // NaN), then, only where that fails somewhere in the wave, element by element.  Once
        // the pre-check has failed, the later tables skip it (data whose bounds are often hit
        // would pay for both).
        const bool chk = a.refine && cA >= 0.f;
        bool exact = !fast;
        if (fast) {
            float amin = fabsf(acc[0][t][0]);
#pragma unroll
            for (int e = 1; e < 16; ++e) amin = __builtin_elementwise_minimum(amin, fabsf(acc[e >> 2][t][e & 3]));
            exact = __any(chk && !(amin > fmaf(rBm, cB, fmaf(rAm, cA, cE))));
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
                    float thr = fmaf(rA[e], cAv, cE);
                    thr = fmaf(rB[e], cB, thr);
                    umask |= !(fabsf(acc[e >> 2][t][e & 3]) > thr) ? (1u << e) : 0u;
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
                const float pv = acc[e >> 2][t][e & 3];
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
                    acc[e >> 2][t][e & 3] = sacc > 0.0 ? 1.f : -1.f;
                }
                ++slot;
            }
        }
        uint32_t f[16];
#pragma unroll
        for (int e = 0; e < 16; ++e) {
            f[e] = (uint32_t)(__ballot(acc[e >> 2][t][e & 3] > 0.f) >> sh);
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
    const int64_t groups = (a.n_tiles_m + 7) / 8;
    const int64_t blocks = groups * 8 * a.n_tiles_n;
    hipLaunchKernelGGL((hash_fp8_kernel<TW>), dim3((unsigned)blocks), dim3(256), 0, s, a);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_convert_fp8(const float* X, int64_t n, int d, int DP, bool vec, uint8_t* Xq, float* rowA,
                              float* rowB, float norm_up, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    const int64_t n16 = (n + 15) / 16 * 16;
    const int64_t blocks = (n16 + 3) / 4;
    if (vec)
        hipLaunchKernelGGL(convert_fp8_kernel<true>, dim3((unsigned)blocks), dim3(256), 0, s, X, n, n16, d, DP, Xq, rowA,
                           rowB, norm_up);
    else
        hipLaunchKernelGGL(convert_fp8_kernel<false>, dim3((unsigned)blocks), dim3(256), 0, s, X, n, n16, d, DP, Xq, rowA,
                           rowB, norm_up);
    return hipGetLastError();
}

hipError_t launch_hash_fp8(const HashArgs& a, int TW, hipStream_t s) {
    switch (TW) {
        case 1: return launch_tw<1>(a, s);
        case 2: return launch_tw<2>(a, s);
        case 4: return launch_tw<4>(a, s);
        case 5: return launch_tw<5>(a, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace ace
