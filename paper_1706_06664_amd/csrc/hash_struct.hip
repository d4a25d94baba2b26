// Structured projections: each bit is the sign of one output of
//   y = H D3 H D2 H D1 [x; 0]        (one block of dp outputs; blocks b = 0 .. B-1)
// with H the dp x dp Sylvester Hadamard matrix (+-1 entries, unnormalised), D random sign
// diagonals and x zero-padded to dp (a power of two >= 64).  Output i of block b is bit
// c = b dp + i, bit k of table j is c = j K + k.  A hash costs 3 B dp log2(dp) additions
// instead of the d K L multiply-adds of a dense W: the fast-transform cost the paper
// states for its hashes (Sec. 2.1, Sec. 3.4).
//
// One wave per row; element e of the transform lives in lane e % 64, register e / 64
// (R = dp / 64 registers).  Butterfly stages of stride s < 64 pair lanes l and l ^ s
// (shuffles); strides >= 64 pair registers inside a lane.
//
// Error bound.  A butterfly stage maps z to (a + b, a - b) pairs: it is sqrt(2) times an
// orthogonal map and each output carries one FP32 rounding (u = 2^-24), so one transform
// of m = log2(dp) stages returns H z with 2-norm error <= g sqrt(dp) |z|, g = m u (1+2u)^m.
// Sign flips are exact.  Carrying that through three rounds:
//   |y_hat - y|_2 <= g dp^1.5 |x|_2 (3 + 4g),
// which bounds every component.  A bit whose |y_hat| is within that bound (plus an
// absolute term for flushed or subnormal intermediates) is queued for the FP64 pass,
// which recomputes sum_t x_t M[c][t] with the dense integer matrix M (exact in FP32), the
// same sum the oracle takes; if the queue is full the wave decides it in place.
#include "ace_internal.h"

namespace ace {

namespace {

template <int R>
__device__ inline void butterflies(float (&v)[R], int lane) {
    // cross-lane strides 1 .. 32
#pragma unroll
    for (int s = 1; s < 64; s <<= 1) {
        const bool hi = (lane & s) != 0;
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const float p = __shfl_xor(v[r], s, 64);
            v[r] = hi ? (p - v[r]) : (v[r] + p);
        }
    }
    // in-lane strides 64 .. dp/2: registers r and r + t
#pragma unroll
    for (int t = 1; t < R; t <<= 1) {
#pragma unroll
        for (int r = 0; r < R; ++r) {
            if (r & t) continue;
            const float x = v[r], y = v[r + t];
            v[r] = x + y;
            v[r + t] = x - y;
        }
    }
}

// Natural layout: bit r of m (this lane's mask) set: negate element e = 64 r + lane
// (branch-free: the bit is moved to the float's sign bit).
template <int R>
__device__ inline void flip(float (&v)[R], u64 m) {
    const uint32_t lo = (uint32_t)m, hi = (uint32_t)(m >> 32);
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const uint32_t bit = r < 32 ? (lo >> r) & 1u : (hi >> (r - 32)) & 1u;
        v[r] = __uint_as_float(__float_as_uint(v[r]) ^ (bit << 31));
    }
}

// Transposed layout (see TR below): register r of lane l holds element
//   e = 64 (l & (R-1)) + ((l & ~(R-1)) | r).
template <int R>
__device__ inline int elem_t(int l, int r) {
    return 64 * (l & (R - 1)) + ((l & ~(R - 1)) | r);
}

// Transposed layout: a lane's R elements are the consecutive bits starting at
// elem_t(lane, 0), a multiple of R, so one aligned 64-bit word of the sign bits holds them.
template <int R>
__device__ inline void flip_t(float (&v)[R], const uint32_t* __restrict__ words, int lane) {
    const int e0 = elem_t<R>(lane, 0);
    const u64 w = reinterpret_cast<const u64*>(words)[e0 >> 6];
    flip<R>(v, w >> (e0 & 63));
}

// Butterflies over the register index (strides 1 .. R/2 of r).
template <int R>
__device__ inline void reg_stages(float (&v)[R]) {
#pragma unroll
    for (int t = 1; t < R; t <<= 1) {
#pragma unroll
        for (int r = 0; r < R; ++r) {
            if (r & t) continue;
            const float x = v[r], y = v[r + t];
            v[r] = x + y;
            v[r + t] = x - y;
        }
    }
}

// Butterflies over lane bits s = R .. 32 (the lane bits the transpose does not move).
template <int R>
__device__ inline void lane_stages_high(float (&v)[R], int lane) {
#pragma unroll
    for (int s = R; s < 64; s <<= 1) {
        const bool hi = (lane & s) != 0;
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const float p = __shfl_xor(v[r], s, 64);
            v[r] = hi ? (p - v[r]) : (v[r] + p);
        }
    }
}

// TR: swap the register index with the low log2(R) lane bits, through LDS (a wave's own
// 65 R floats): (lane l, reg r) -> (lane (l & ~(R-1)) | r, reg l & (R-1)).  It is its own
// inverse.  The word of (l, r) is r * 65 + l, so both the stores and the loads of one
// instruction touch 64 distinct banks.
template <int R>
__device__ inline void transpose(float (&v)[R], float* __restrict__ T, int lane) {
    __builtin_amdgcn_sched_barrier(0);   // keep each phase's live values to its own R registers
#pragma unroll
    for (int r = 0; r < R; ++r) T[r * 65 + lane] = v[r];
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    const int hi = lane & ~(R - 1), lo = lane & (R - 1);
#pragma unroll
    for (int r = 0; r < R; ++r) v[r] = T[lo * 65 + (hi | r)];
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    __builtin_amdgcn_sched_barrier(0);
}

// Masks of one row: bit c % 64 of word c / 64 (sign bits, then uncertain bits).
// TRANS: for R >= 8 the transform moves the register bits and the low lane bits through
// LDS transposes instead of shuffling across lanes (three rounds, four transposes).
template <int R, bool TRANS>
__global__ __launch_bounds__(256) void hash_struct_kernel(const HashArgs a) {
    extern __shared__ u64 masks[];          // per wave: 2 * nw mask words, then 65 R floats
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int dp = 64 * R;
    const int KL = a.K * a.L;
    const int nw = a.nblk * R;              // 64-bit words per row
    const size_t wave_words = 2 * (size_t)nw + (TRANS ? (65 * R + 1) / 2 : 0);
    u64* bits = masks + (size_t)wave * wave_words;
    u64* unc = bits + nw;
    float* Tl = reinterpret_cast<float*>(unc + nw);
    const uint32_t kmask = (a.K >= 16) ? 0xFFFFu : ((1u << a.K) - 1u);
    const int64_t rows_per_block = 4 * (int64_t)a.rows_per_wave;
    uint32_t n_ref = 0, n_flip = 0, n_unc = 0;
    const int64_t nv = a.n_dev ? *a.n_dev : a.n;   // real rows

    for (int rw = 0; rw < a.rows_per_wave; ++rw) {
        const int64_t row = (int64_t)blockIdx.x * rows_per_block + (int64_t)wave * a.rows_per_wave + rw;
        if (row >= nv) break;   // uniform over the wave
        const float* xr = a.X + row * (int64_t)a.d;
        float E = 0.f;
        for (int b = 0; b < a.nblk; ++b) {
            float v[R];
            {
                // The row again for every block, through a buffer resource limited to its d
                // floats: elements e >= d read as 0 (the zero padding) with no per-element test.
                const __amdgpu_buffer_rsrc_t rs =
                    __builtin_amdgcn_make_buffer_rsrc((void*)xr, (short)0, a.d * 4, 0x00020000);
#pragma unroll
                for (int r = 0; r < R; ++r)
                    v[r] = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(rs, (64 * r + lane) * 4, 0, 0));
            }
            if (b == 0) {   // bound of this row: gx |x|_2 + eps_abs (FP64 norm, rounded up)
                double ss = 0.0;
#pragma unroll
                for (int r = 0; r < R; ++r) ss += (double)v[r] * (double)v[r];
                for (int off = 32; off > 0; off >>= 1) ss += __shfl_xor(ss, off, 64);
                E = (float)((double)a.gx * sqrt(ss) * (1.0 + 0x1p-20)) + a.eps_abs;
            }
            __builtin_amdgcn_sched_barrier(0);
            const uint32_t* sg = a.sgn + (size_t)b * 3 * (dp / 32);
            const u64* sl = a.sgn_lane + (size_t)b * 3 * 64 + lane;   // bit r: element 64 r + lane
            if (TRANS) {
                // sign-and-transform pass 1 (natural -> transposed), pass 2 (transposed -> natural),
                // pass 3 (natural -> transposed), then back to the natural layout
                flip<R>(v, sl[0]);
                reg_stages<R>(v);
                transpose<R>(v, Tl, lane);
                reg_stages<R>(v);
                lane_stages_high<R>(v, lane);
                flip_t<R>(v, sg + dp / 32, lane);
                reg_stages<R>(v);
                transpose<R>(v, Tl, lane);
                reg_stages<R>(v);
                lane_stages_high<R>(v, lane);
                flip<R>(v, sl[128]);
                reg_stages<R>(v);
                transpose<R>(v, Tl, lane);
                reg_stages<R>(v);
                lane_stages_high<R>(v, lane);
                transpose<R>(v, Tl, lane);
                __builtin_amdgcn_sched_barrier(0);
            } else {
                flip<R>(v, sl[0]);
                butterflies<R>(v, lane);
                flip<R>(v, sl[64]);
                butterflies<R>(v, lane);
                flip<R>(v, sl[128]);
                butterflies<R>(v, lane);
            }
            __builtin_amdgcn_sched_barrier(0);
            // Masks of register r end up in lane r (each ballot is consumed at once), then
            // lanes 0 .. R-1 store them together.
            u64 my_bits = 0, my_unc = 0;
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const int c = b * dp + 64 * r + lane;
                const bool valid = c < KL;
                const u64 bm = __ballot(valid && v[r] > 0.f);
                const u64 um = a.refine ? __ballot(valid && !(fabsf(v[r]) > E)) : 0ull;   // NaN is uncertain
                my_bits = lane == r ? bm : my_bits;
                my_unc = lane == r ? um : my_unc;
            }
            if (lane < R) {
                bits[b * R + lane] = my_bits;
                unc[b * R + lane] = my_unc;
            }
        }
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");

        // Uncertain bits: queue them (one atomic per wave and row) or count them (refine = 2).
        uint32_t mine = 0;
        for (int i = lane; i < nw; i += 64) mine += (uint32_t)__popcll(unc[i]);
        if (a.refine == 2) {
            n_unc += mine;
        } else if (__any(mine != 0)) {
            uint32_t incl = mine;
#pragma unroll
            for (int off = 1; off < 64; off <<= 1) {
                const uint32_t t = __shfl_up(incl, off, 64);
                if (lane >= off) incl += t;
            }
            const uint32_t total = __shfl(incl, 63, 64);
            u64 base = 0;
            if (lane == 0) base = atomicAdd(a.list_count, (u64)total);
            base = __shfl(base, 0, 64);
            u64 slot = base + (incl - mine);
            for (int i = lane; i < nw; i += 64) {
                u64 um = unc[i];
                while (um) {
                    const int bpos = __ffsll((long long)um) - 1;
                    um &= um - 1;
                    const int c = 64 * i + bpos;
                    const int cp = (c / a.K) * KPAD + (c % a.K);
                    const bool raw = (bits[i] >> bpos) & 1ull;
                    if (slot < a.list_cap) {
                        a.list[slot] = (u64)(uint32_t)row | ((u64)cp << 32) | (raw ? (1ull << 63) : 0ull);
                    } else {
                        // Queue full: decide here (same FP64 sum as the FP64 pass).
                        const float* wr = a.Wt + (int64_t)cp * a.DP;
                        double s = 0.0;
                        for (int t = 0; t < a.d; ++t) s += (double)xr[t] * (double)wr[t];
                        mark_refined(a, row, cp);
                        n_ref += 1u;
                        n_flip += ((s > 0.0) != raw) ? 1u : 0u;
                        if (s > 0.0) bits[i] |= 1ull << bpos;
                        else bits[i] &= ~(1ull << bpos);
                    }
                    ++slot;
                }
            }
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        }

        // Codes: lane t packs tables t, t + 64, ...
        for (int j = lane; j < a.L; j += 64) {
            const int c0 = j * a.K;
            const int i0 = c0 >> 6, o = c0 & 63;
            u64 w = bits[i0] >> o;
            if (o + a.K > 64) w |= bits[i0 + 1] << (64 - o);
            a.codes[(int64_t)j * a.ldc + row] = (uint16_t)((uint32_t)w & kmask);
        }
        __builtin_amdgcn_wave_barrier();
    }
    if (__any(n_ref != 0 || n_unc != 0)) {
        uint32_t r = n_ref, f = n_flip, uc = n_unc;
        for (int off = 32; off > 0; off >>= 1) {
            r += __shfl_xor(r, off, 64);
            f += __shfl_xor(f, off, 64);
            uc += __shfl_xor(uc, off, 64);
        }
        if (lane == 0) {
            if (r) atomicAdd(&a.counters[0], (u64)r);
            if (f) atomicAdd(&a.counters[1], (u64)f);
            if (uc) atomicAdd(&a.counters[2], (u64)uc);
        }
    }
}

}  // namespace

hipError_t init_struct_attributes() {
    const void* fns[] = {reinterpret_cast<const void*>(&hash_struct_kernel<1, false>),
                         reinterpret_cast<const void*>(&hash_struct_kernel<2, false>),
                         reinterpret_cast<const void*>(&hash_struct_kernel<4, false>),
                         reinterpret_cast<const void*>(&hash_struct_kernel<8, true>),
                         reinterpret_cast<const void*>(&hash_struct_kernel<16, true>),
                         reinterpret_cast<const void*>(&hash_struct_kernel<32, true>),
                         reinterpret_cast<const void*>(&hash_struct_kernel<64, true>)};
    for (const void* f : fns) {
        const hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, 128 * 1024);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_hash_struct(const HashArgs& a, hipStream_t s) {
    if (a.n <= 0) return hipSuccess;
    const int R = a.dp / 64;
    const int64_t rows_per_block = 4 * (int64_t)a.rows_per_wave;
    const int64_t nb = (a.n + rows_per_block - 1) / rows_per_block;
    const bool trans = R >= 8;
    const size_t wave_words = 2 * (size_t)a.nblk * R + (trans ? (65 * (size_t)R + 1) / 2 : 0);
    const size_t lds = sizeof(u64) * wave_words * 4;
    if (lds > 128 * 1024) return hipErrorInvalidValue;   // K L <= 32768 at dp = 4096
    switch (R) {
#define ACE_STRUCT_CASE(RR)                                                                                      \
    case RR:                                                                                                     \
        hipLaunchKernelGGL((hash_struct_kernel<RR, (RR >= 8)>), dim3((unsigned)nb), dim3(256), lds, s, a);      \
        break;
        ACE_STRUCT_CASE(1)
        ACE_STRUCT_CASE(2)
        ACE_STRUCT_CASE(4)
        ACE_STRUCT_CASE(8)
        ACE_STRUCT_CASE(16)
        ACE_STRUCT_CASE(32)
        ACE_STRUCT_CASE(64)
#undef ACE_STRUCT_CASE
        default:
            return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace ace
