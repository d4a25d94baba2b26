// The FP64 pass over the queued projections (Sec. 2.1 signs, decided exactly where the
// low-precision projection could not decide them).  Entry = row | column << 32 | raw bit
// << 63.  Every kernel here computes the FP64 sum over ascending t from the FP32 inputs
// (products of FP32 values are exact in FP64, so this is the value a plain FP64 loop
// produces) and sets or clears the code bit with a 32-bit atomic on the word holding the
// code (the workspace is padded so that word never leaves it); `refined` (optional, same
// layout as the codes) gets the bit marked.
#include "ace_internal.h"

namespace ace {

namespace {

typedef float f4 __attribute__((ext_vector_type(4)));

__device__ inline uint32_t wave_sum_u32(uint32_t v) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// One thread per entry.
template <bool VEC>
__global__ __launch_bounds__(256) void refine_kernel(const RefineArgs a) {
    const u64 n_ent = min(*a.list_count, a.list_cap);
    if (a.clear_next && blockIdx.x == 0 && threadIdx.x == 0) *a.clear_next = 0ull;
    uint32_t n_ref = 0, n_flip = 0;
    for (u64 i = (u64)blockIdx.x * blockDim.x + threadIdx.x; i < n_ent; i += (u64)gridDim.x * blockDim.x) {
        const u64 e = a.list[i];
        const int64_t row = (int64_t)(e & 0xFFFFFFFFull);
        const int cp = (int)((e >> 32) & 0xFFFFu);
        const bool raw = (e >> 63) != 0;
        const float* xr = a.X + row * (int64_t)a.d;
        const float* wr = a.Wt + (int64_t)cp * a.DP;
        double s = 0.0;
        int u = 0;
        if (VEC) {
            // 16-byte loads, four in flight; the additions still run in ascending t.
            for (; u + 16 <= a.d; u += 16) {
                const f4 x0 = *reinterpret_cast<const f4*>(xr + u), w0 = *reinterpret_cast<const f4*>(wr + u);
                const f4 x1 = *reinterpret_cast<const f4*>(xr + u + 4), w1 = *reinterpret_cast<const f4*>(wr + u + 4);
                const f4 x2 = *reinterpret_cast<const f4*>(xr + u + 8), w2 = *reinterpret_cast<const f4*>(wr + u + 8);
                const f4 x3 = *reinterpret_cast<const f4*>(xr + u + 12), w3 = *reinterpret_cast<const f4*>(wr + u + 12);
#pragma unroll
                for (int q = 0; q < 4; ++q) s += (double)x0[q] * (double)w0[q];
#pragma unroll
                for (int q = 0; q < 4; ++q) s += (double)x1[q] * (double)w1[q];
#pragma unroll
                for (int q = 0; q < 4; ++q) s += (double)x2[q] * (double)w2[q];
#pragma unroll
                for (int q = 0; q < 4; ++q) s += (double)x3[q] * (double)w3[q];
            }
        }
        for (; u < a.d; ++u) s += (double)xr[u] * (double)wr[u];
        const bool bit = s > 0.0;
        const int table = cp >> 4, k = cp & 15;
        if (table < a.L && k < a.K) {
            const size_t idx = (size_t)table * a.ldc + row;
            const uintptr_t addr = reinterpret_cast<uintptr_t>(a.codes + idx);
            uint32_t* word = reinterpret_cast<uint32_t*>(addr & ~(uintptr_t)3);
            const uint32_t m = 1u << (k + ((addr & 2) ? 16 : 0));
            if (bit != raw) {
                if (bit) atomicOr(word, m);
                else atomicAnd(word, ~m);
            }
            if (a.refined) {
                const uintptr_t ra = reinterpret_cast<uintptr_t>(a.refined + idx);
                atomicOr(reinterpret_cast<uint32_t*>(ra & ~(uintptr_t)3), 1u << (k + ((ra & 2) ? 16 : 0)));
            }
            n_ref += 1u;
            n_flip += (bit != raw) ? 1u : 0u;
        }
    }
    const uint32_t r = wave_sum_u32(n_ref), f = wave_sum_u32(n_flip);
    if ((threadIdx.x & 63) == 0 && r) {
        atomicAdd(&a.counters[0], (u64)r);
        if (f) atomicAdd(&a.counters[1], (u64)f);
    }
}

// FP64 pass, staged variant (16-byte aligned rows, d % 4 == 0).  A wave takes 64 queue
// entries, one per lane, and walks k in chunks of 32: the wave loads the chunk of every
// entry's row and column with 16-byte loads (eight lanes per entry, so each load
// instruction reads eight whole 128-byte segments), parks them in LDS, and then every lane
// runs its entry's FP64 sum over the chunk in ascending t.  The sum and the bit patch are
// those of refine_kernel; only the memory access pattern differs.
// Each wave stages into its own LDS slice, so a wave-level ordering point suffices: LDS
// operations of one wave complete in issue order.
__device__ inline void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}
constexpr int RC = 32;        // k per chunk
constexpr int RS = RC + 1;    // LDS row stride in floats (lane e reads row e: distinct banks)

__global__ __launch_bounds__(256, 2) void refine_staged_kernel(const RefineArgs a) {
    __shared__ float xs[4][64 * RS], ws[4][64 * RS];
    const u64 n_ent = min(*a.list_count, a.list_cap);
    if (a.clear_next && blockIdx.x == 0 && threadIdx.x == 0) *a.clear_next = 0ull;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int d = a.d;
    float* xw = xs[wave];
    float* ww = ws[wave];
    uint32_t n_ref = 0, n_flip = 0;
    for (u64 g0 = (u64)blockIdx.x * 256; g0 < n_ent; g0 += (u64)gridDim.x * 256) {
        const u64 i = g0 + (u64)threadIdx.x;
        const bool ok = i < n_ent;
        const u64 e = ok ? a.list[i] : 0ull;
        const int64_t row = (int64_t)(e & 0xFFFFFFFFull);
        const int cp = (int)((e >> 32) & 0xFFFFu);
        double s = 0.0;
        // Lane l stages 4 values of entry 8j + l/8 (j = 0..7) at t0 + 4 (l % 8); the next
        // chunk's loads are issued before the current chunk is summed.
        const int q = 4 * (lane & 7);
        const float* xr[8];
        const float* wr[8];
        bool eok[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const int ee = 8 * j + (lane >> 3);
            const int64_t er = __shfl(row, ee, 64);
            const int ec = __shfl(cp, ee, 64);
            eok[j] = g0 + (u64)(64 * wave + ee) < n_ent;
            xr[j] = a.X + er * (int64_t)d + q;
            wr[j] = a.Wt + (int64_t)ec * a.DP + q;
        }
        f4 xv[8], wv[8];
        auto load = [&](int t0) {
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                xv[j] = f4{0.f, 0.f, 0.f, 0.f};
                wv[j] = f4{0.f, 0.f, 0.f, 0.f};
                if (eok[j]) {
                    if (t0 + q + 4 <= d) {
                        xv[j] = *reinterpret_cast<const f4*>(xr[j] + t0);
                    } else {
#pragma unroll
                        for (int u = 0; u < 4; ++u) xv[j][u] = (t0 + q + u < d) ? xr[j][t0 + u] : 0.f;
                    }
                    // W^T rows are zero-padded to DP, a multiple of the chunk size.
                    wv[j] = *reinterpret_cast<const f4*>(wr[j] + t0);
                }
            }
        };
        load(0);
        for (int t0 = 0; t0 < d; t0 += RC) {
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                const int ee = 8 * j + (lane >> 3);
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    xw[ee * RS + q + u] = xv[j][u];
                    ww[ee * RS + q + u] = wv[j][u];
                }
            }
            if (t0 + RC < d) load(t0 + RC);
            wave_sync();
            // Past d the staged values are zeros: adding an exact zero leaves the sum's
            // value unchanged (at most -0 becomes +0, which is not > 0 either way).
#pragma unroll 8
            for (int t = 0; t < RC; ++t) s = fma((double)xw[lane * RS + t], (double)ww[lane * RS + t], s);
            wave_sync();
        }
        if (ok) {
            const bool raw = (e >> 63) != 0;
            const bool bit = s > 0.0;
            const int table = cp >> 4, k = cp & 15;
            if (table < a.L && k < a.K) {
                const size_t idx = (size_t)table * a.ldc + row;
                const uintptr_t addr = reinterpret_cast<uintptr_t>(a.codes + idx);
                uint32_t* word = reinterpret_cast<uint32_t*>(addr & ~(uintptr_t)3);
                const uint32_t m = 1u << (k + ((addr & 2) ? 16 : 0));
                if (bit != raw) {
                    if (bit) atomicOr(word, m);
                    else atomicAnd(word, ~m);
                }
                if (a.refined) {
                    const uintptr_t ra = reinterpret_cast<uintptr_t>(a.refined + idx);
                    atomicOr(reinterpret_cast<uint32_t*>(ra & ~(uintptr_t)3), 1u << (k + ((ra & 2) ? 16 : 0)));
                }
                n_ref += 1u;
                n_flip += (bit != raw) ? 1u : 0u;
            }
        }
    }
    const uint32_t r = wave_sum_u32(n_ref), f = wave_sum_u32(n_flip);
    if (lane == 0 && r) {
        atomicAdd(&a.counters[0], (u64)r);
        if (f) atomicAdd(&a.counters[1], (u64)f);
    }
}

}  // namespace

int cu_count() {
    static int cus[64] = {0};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
    if (cus[dev] == 0) {
        int n = 0;
        if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n <= 0) n = 256;
        cus[dev] = n;
    }
    return cus[dev];
}

hipError_t launch_refine(const RefineArgs& a, int64_t max_entries, bool vec, hipStream_t s) {
    int64_t blocks = (max_entries + 255) / 256;
    // Staging pays once rows are long enough for the chunk loop to be worth its barriers
    // (at d = 120 it already takes 0.018 against 0.021 ms for about 2,500 entries).
    if (vec && a.d >= 64 && a.DP % RC == 0) {
        const int64_t resident = (int64_t)cu_count() * 2;
        if (blocks > resident) blocks = resident;
        if (blocks < 1) blocks = 1;
        hipLaunchKernelGGL(refine_staged_kernel, dim3((unsigned)blocks), dim3(256), 0, s, a);
        return hipGetLastError();
    }
    if (blocks > 4096) blocks = 4096;
    if (blocks < 1) blocks = 1;
    if (vec)
        hipLaunchKernelGGL(refine_kernel<true>, dim3((unsigned)blocks), dim3(256), 0, s, a);
    else
        hipLaunchKernelGGL(refine_kernel<false>, dim3((unsigned)blocks), dim3(256), 0, s, a);
    return hipGetLastError();
}

}  // namespace ace
