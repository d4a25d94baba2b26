// SRP hashing on FP32 MFMA (Sec. 2.1 signed random projections, Sec. 3.2 K-bit codes).
//
// One launch computes P = X W for a chunk of rows on v_mfma_f32_16x16x4f32 and never
// writes P: the epilogue turns each 16-column output tile (one table) into bits
// (p > 0) and packs the 16 bits of each row into a uint16 code.  Every projection
// whose FP32 value lies inside its error bound is queued (one atomic per wave) and
// decided by refine_kernel in FP64; if the queue is full the epilogue decides it
// in place.
//
// Error bound of an FP32 projection (Higham, Accuracy and Stability of Numerical
// Algorithms, 2nd ed., Sec. 3.1): if every term x_t w_t passes through at most h
// roundings of relative size u, then
//   |p32 - p| <= gamma_h(u) sum_t |x_t w_t| <= gamma_h(u) ||x|| ||w||.
// The host passes gamma_h(u) for the context's error model: h = DP + 4 with
// u = 2^-24 (exact products, one round-to-nearest per product added, as measured on
// gfx950), or h = 2 DP + 8 with u = 2^-23 (any instruction losing up to 6 units of
// 2^-23), plus an absolute term for flushed subnormals.  Outside the bound the sign
// of p32 is the sign of p; inside it the FP64 sum over ascending t is taken (products
// of FP32 values are exact in FP64, so this is the same value a plain FP64 loop
// produces).
//
// Two kernels.  Rows that are 16-byte aligned with d % 4 == 0 go to the direct kernel
// (operands loaded straight into registers, persistent grid); other inputs go to the LDS
// kernel.  LDS kernel tiling: 256 threads = 4 waves as 2 (rows) x 2 (columns).  A
// workgroup tile is 128 rows x 2*TW tables (32*TW padded columns); each wave holds 64
// rows x TW tables = 4 x TW MFMA tiles of 16x16.  The contraction runs in chunks of 32
// through LDS; both operands are stored k-contiguous so each lane reads one float4 per
// 16-wide k block and feeds four MFMAs with it.
#include <type_traits>

#include "ace_internal.h"

namespace ace {

namespace {

constexpr int BM = 128;
constexpr int BK = 32;
constexpr int LDSW = BK + 4;  // padded LDS row stride (floats)
// Direct kernel: 16-row blocks per wave and resident waves per SIMD (its register budget).
constexpr int DIRECT_RB = 4;
constexpr int DIRECT_WAVES = 2;

typedef float f4 __attribute__((ext_vector_type(4)));

// Sign packing.  Lane l stores row rho = l & 15 of 16-row tile l >> 4.  Tile b's ballot of
// accumulator element r holds row 4g + r in bits 16g .. 16g + 15 (lane 16g + c holds column
// c), so lane l needs ballot pick = 4 (l >> 4) + (l & 3) shifted right by 16 ((l & 15) >> 2).
// f[e] is ballot e already shifted by the lane's amount; a select tree over the bits of pick
// keeps the lane's own (masks, not branches or a switch).  Lanes with pick >= N get an unused
// value.
template <int N>
__device__ inline uint32_t pick_code(uint32_t (&f)[N], int pick) {
#pragma unroll
    for (int w = 1; w < N; w <<= 1) {
        const uint32_t m = 0u - (uint32_t)((pick & w) != 0);
#pragma unroll
        for (int i = 0; i + w < N; i += 2 * w) f[i] = (f[i + w] & m) | (f[i] & ~m);
    }
    return f[0];
}

__device__ inline uint32_t wave_sum_u32(uint32_t v) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Epilogue shared by the projection kernels.  acc[b][t] (b < RB) is the 16x16 MFMA tile of
// rows rbase + 16b .. and padded columns cbase + 16t ..; lane l holds rows 16b + 4(l/16) + r
// (r = 0..3) of column l%16; only tables t with bit t of tmask are finished here.
// rbnd[4b + r] is the row bound factor of that row and wcol[t]
// the column factor of this lane's column in tile t.  Projections inside their bound are
// queued for the FP64 pass (or decided here when the queue is full); each 16-column tile
// is one table, whose bits are gathered with ballots and stored as one uint16 per row.
template <int TW, int RB>
__device__ inline void sign_epilogue(const HashArgs& a, f4 (&acc)[RB][TW], const float (&rbnd)[4 * RB],
                                     const float (&wcol)[TW], int64_t rbase, int cbase, int64_t nv, int lane,
                                     uint32_t tmask = ~0u) {
    const int kin = lane >> 4, cl = lane & 15;
    // Rows past the batch's real rows (only the last row tile has any) take no bits: their
    // accumulators become +inf, outside every bound, and their codes are not stored.
    if (rbase + 16 * RB > nv) {
#pragma unroll
        for (int e = 0; e < 4 * RB; ++e)
            if (rbase + 16 * (e >> 2) + 4 * kin + (e & 3) >= nv) {
#pragma unroll
                for (int t = 0; t < TW; ++t) acc[e >> 2][t][e & 3] = __builtin_inff();
            }
    }
    const uint32_t kmask = (a.K >= 16) ? 0xFFFFu : ((1u << a.K) - 1u);
    const int64_t orow = rbase + lane;  // the row whose codes this lane stores (lanes < 16 RB)
    const int pick = 4 * kin + (lane & 3), sh = 16 * ((lane & 15) >> 2);
    // The largest of this lane's row bound factors (the maximum keeps a NaN).
    float rbmax = rbnd[0];
#pragma unroll
    for (int e = 1; e < 4 * RB; ++e) rbmax = __builtin_elementwise_maximum(rbmax, rbnd[e]);
    uint32_t n_ref = 0, n_flip = 0, n_unc = 0;                // projections decided in place (queue full)
    bool fast = true;  // wave-uniform
#pragma unroll
    for (int t = 0; t < TW; ++t) {
        if (!((tmask >> t) & 1u)) continue;  // a table another wave finishes
        const int table = (cbase >> 4) + t;
        const int cp = cbase + t * 16 + cl;
        const float wbv = wcol[t];
        const bool chk = a.refine && wbv >= 0.f;
        // Is any accumulator element of this lane inside its bound?  (NaN is uncertain too.)
        // First against the lane's largest bound (one comparison of the smallest |acc|; the
        // minimum keeps a NaN), then, only where that fails somewhere in the wave, element by
        // element.  Once the pre-check has failed, the tile's later tables skip it (data whose
        // bounds are often hit would pay for both).
        bool exact = !fast;
        if (fast) {
            float amin = fabsf(acc[0][t][0]);
#pragma unroll
            for (int e = 1; e < 4 * RB; ++e) amin = __builtin_elementwise_minimum(amin, fabsf(acc[e >> 2][t][e & 3]));
            exact = __any(chk && !(amin > fmaf(rbmax, wbv, a.eps_abs)));
            fast = !exact;
        }
        bool unc = false;
        if (exact) {
            // (The empty asm keeps these 4 RB bounds from being computed ahead of the test.)
            float wv = wbv;
            asm volatile("" : "+v"(wv));
#pragma unroll
            for (int e = 0; e < 4 * RB; ++e) unc |= !(fabsf(acc[e >> 2][t][e & 3]) > fmaf(rbnd[e], wv, a.eps_abs));
            unc = unc && chk;
        }
        uint32_t code = 0;
        if (a.refine != 2 && !__any(unc)) {
            // Common case: the signs stand; ballots straight from the accumulators.
            uint32_t f[4 * RB];
#pragma unroll
            for (int e = 0; e < 4 * RB; ++e) {
                f[e] = (uint32_t)(__ballot(acc[e >> 2][t][e & 3] > 0.f) >> sh);
                // Shift each ballot as it is taken: selecting the unshifted scalar pairs
                // first would cost two vector selects (and copies) per pair.
                asm("" : "+v"(f[e]));
            }
            code = pick_code(f, pick);
        } else {
            // Bit e of umask: accumulator element e lies inside its bound.
            uint32_t umask = 0;
#pragma unroll
            for (int e = 0; e < 4 * RB; ++e) {
                const float thr = fmaf(rbnd[e], wbv, a.eps_abs);
                umask |= (chk && !(fabsf(acc[e >> 2][t][e & 3]) > thr)) ? (1u << e) : 0u;
            }
            if (a.refine == 2) {
                n_unc += __popc(umask);  // count only: the raw signs stand
                umask = 0;
            }
            // Rare: queue each uncertain (row, column) for the FP64 pass, one atomic per wave;
            // bit e of pos is the sign of element e (patched where decided in place).
            uint32_t pos = 0;
#pragma unroll
            for (int e = 0; e < 4 * RB; ++e) pos |= (acc[e >> 2][t][e & 3] > 0.f) ? (1u << e) : 0u;
            const uint32_t mine = __popc(umask);
            uint32_t incl = mine;
#pragma unroll
            for (int off = 1; off < 64; off <<= 1) {
                const uint32_t v = __shfl_up(incl, off, 64);
                if (lane >= off) incl += v;
            }
            const uint32_t total = __shfl(incl, 63, 64);
            u64 base = 0;
            if (total != 0) {
                if (lane == 0) base = atomicAdd(a.list_count, (u64)total);
                base = __shfl(base, 0, 64);
            }
            u64 slot = base + (incl - mine);
            uint32_t todo = umask;
            while (todo) {
                const int e = __builtin_ctz(todo);
                todo &= todo - 1u;
                const int64_t grow = rbase + 16 * (e >> 2) + 4 * kin + (e & 3);
                const bool raw = (pos >> e) & 1u;
                if (slot < a.list_cap) {
                    a.list[slot] = (u64)(uint32_t)grow | ((u64)cp << 32) | (raw ? (1ull << 63) : 0ull);
                } else {
                    // Queue full: decide here (same FP64 sum as the FP64 pass).
                    const float* xr = a.X + grow * (int64_t)a.d;
                    const float* wr = a.Wt + (int64_t)cp * a.DP;
                    double sacc = 0.0;
                    for (int u = 0; u < a.d; ++u) sacc += (double)xr[u] * (double)wr[u];
                    mark_refined(a, grow, cp);
                    n_ref += 1u;
                    n_flip += ((sacc > 0.0) != raw) ? 1u : 0u;
                    pos = sacc > 0.0 ? (pos | (1u << e)) : (pos & ~(1u << e));
                }
                ++slot;
            }
            uint32_t f[4 * RB];
#pragma unroll
            for (int e = 0; e < 4 * RB; ++e) f[e] = (uint32_t)(__ballot((pos >> e) & 1u) >> sh);
            code = pick_code(f, pick);
        }
        if (table < a.L && lane < 16 * RB && orow < nv) a.codes[(int64_t)table * a.ldc + orow] = (uint16_t)(code & kmask);
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

template <int TW, bool VEC>
__global__ __launch_bounds__(256) void hash_fp32_kernel(const HashArgs a) {
    constexpr int NB = 32 * TW;
    __shared__ float As[BM * LDSW];
    __shared__ float Bs[NB * LDSW];
    __shared__ float rowb[BM];

    // Workgroups are dispatched round-robin over the 8 XCDs (block b runs on XCD b % 8).
    // Give the blocks of one XCD all column tiles of the same row tile, back to back,
    // so that XCD's L2 serves the repeated reads of the X tile.
    const int64_t bid = blockIdx.x;
    const int64_t xcd = bid & 7, local = bid >> 3;
    const int64_t tile_n = local % a.n_tiles_n;
    const int64_t tile_m = (local / a.n_tiles_n) * 8 + xcd;
    if (tile_m >= a.n_tiles_m) return;

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave >> 1, wn = wave & 1;
    const int64_t row0 = tile_m * BM;
    const int64_t nv = a.n_dev ? *a.n_dev : a.n;   // real rows (loads stay within the n rows)
    const int col0 = (int)tile_n * NB;

    f4 acc[4][TW];
#pragma unroll
    for (int b = 0; b < 4; ++b)
#pragma unroll
        for (int t = 0; t < TW; ++t) acc[b][t] = f4{0.f, 0.f, 0.f, 0.f};

    // A-tile role: thread -> row lr, 16 consecutive k at lk.
    const int lr = tid >> 1, lk = (tid & 1) * 16;
    const int64_t grow_ld = row0 + lr;
    const bool row_ok = grow_ld < a.n;
    const float* xrow = a.X + (row_ok ? grow_ld : 0) * (int64_t)a.d;
    double ss = 0.0;

    // Column bound factors of this wave's tables (read early; used in the epilogue).
    float wcol[TW];
#pragma unroll
    for (int t = 0; t < TW; ++t) wcol[t] = a.wb[col0 + (wn * TW + t) * 16 + (lane & 15)];

    for (int k0 = 0; k0 < a.d; k0 += BK) {
        float v[16];
        if (VEC) {
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int k = k0 + lk + 4 * q;
                f4 t = f4{0.f, 0.f, 0.f, 0.f};
                if (row_ok && k < a.d) t = *reinterpret_cast<const f4*>(xrow + k);
                v[4 * q + 0] = t[0];
                v[4 * q + 1] = t[1];
                v[4 * q + 2] = t[2];
                v[4 * q + 3] = t[3];
            }
        } else {
#pragma unroll
            for (int e = 0; e < 16; ++e) {
                const int k = k0 + lk + e;
                v[e] = (row_ok && k < a.d) ? xrow[k] : 0.f;
            }
        }
#pragma unroll
        for (int e = 0; e < 16; ++e) ss += (double)v[e] * (double)v[e];
#pragma unroll
        for (int q = 0; q < 4; ++q)
            *reinterpret_cast<f4*>(As + lr * LDSW + lk + 4 * q) =
                f4{v[4 * q], v[4 * q + 1], v[4 * q + 2], v[4 * q + 3]};
        // B tile: NB columns x 32 k as float4 quads; W is zero-padded to DP and NP.
#pragma unroll
        for (int s = 0; s < TW; ++s) {
            const int q = tid + 256 * s;
            const int col = q >> 3, kq = (q & 7) * 4;
            const f4 t = *reinterpret_cast<const f4*>(a.Wt + (int64_t)(col0 + col) * a.DP + k0 + kq);
            *reinterpret_cast<f4*>(Bs + col * LDSW + kq) = t;
        }
        __syncthreads();
#pragma unroll
        for (int kb = 0; kb < BK; kb += 16) {
            // MFMA step s of this block uses k = kb + 4*(lane>>4) + s on both operands.
            f4 af[4];
#pragma unroll
            for (int b = 0; b < 4; ++b)
                af[b] = *reinterpret_cast<const f4*>(As + (wm * 64 + 16 * b + (lane & 15)) * LDSW + kb +
                                                     4 * (lane >> 4));
#pragma unroll
            for (int t = 0; t < TW; ++t) {
                const f4 bf = *reinterpret_cast<const f4*>(Bs + ((wn * TW + t) * 16 + (lane & 15)) * LDSW +
                                                           kb + 4 * (lane >> 4));
#pragma unroll
                for (int b = 0; b < 4; ++b) {
                    acc[b][t] = __builtin_amdgcn_mfma_f32_16x16x4f32(af[b][0], bf[0], acc[b][t], 0, 0, 0);
                    acc[b][t] = __builtin_amdgcn_mfma_f32_16x16x4f32(af[b][1], bf[1], acc[b][t], 0, 0, 0);
                    acc[b][t] = __builtin_amdgcn_mfma_f32_16x16x4f32(af[b][2], bf[2], acc[b][t], 0, 0, 0);
                    acc[b][t] = __builtin_amdgcn_mfma_f32_16x16x4f32(af[b][3], bf[3], acc[b][t], 0, 0, 0);
                }
            }
        }
        __syncthreads();
    }

    // Row bound factor: gx * ||x|| (FP64 sum of squares, rounded up by a relative 2^-20).
    ss += __shfl_xor(ss, 1, 64);
    if ((tid & 1) == 0) rowb[lr] = (float)(a.gx * sqrt(ss) * (1.0 + 0x1p-20));
    __syncthreads();

    // This lane's 16 accumulator rows: wm*64 + 16b + 4*kin + r (b, r = 0..3), index e = 4b + r.
    const int kin = lane >> 4;
    float rbnd[16];
#pragma unroll
    for (int b = 0; b < 4; ++b) {
        const f4 v = *reinterpret_cast<const f4*>(rowb + wm * 64 + 16 * b + 4 * kin);
#pragma unroll
        for (int r = 0; r < 4; ++r) rbnd[4 * b + r] = v[r];
    }
    sign_epilogue<TW, 4>(a, acc, rbnd, wcol, row0 + wm * 64, col0 + wn * TW * 16, nv, lane);
}

// Direct-operand variant (d % 4 == 0, 16-byte aligned rows): each wave loads its MFMA
// operands from global memory straight into registers, one 16-byte load per lane for each
// 16-row (or 16-column) tile and 16-wide k block, issued one block ahead of the MFMAs that
// use them.  No LDS and no barriers: the four waves of a workgroup run on their own, and
// the two waves that share rows (or columns) share them through the CU's L1 and the XCD's
// L2.  Lane l feeds k = kb + 4(l/16) + s to MFMA step s, for rows (A) and columns (B)
// alike.  The last partial block of d takes only the steps it needs: 2 for 8 remaining
// k (k = kb + 2(l/16) + s), 1 for 4 (k = kb + l/16); with 12 the fourth k group is zero.
// Rows past n read as zero (range-checked buffer loads over the wave's rows).
//
// The grid is persistent: workgroup g takes tile slots g, g + G, g + 2G, ... (G, the grid
// size, is a multiple of 8, so every slot of a workgroup maps to the same XCD), and the
// rows of the first k block of a wave's next tile are loaded before the sign epilogue of
// its current one, so that load's latency is spent on the epilogue.
//
// Tiling: 4 waves as 2 (rows) x 2 (columns); a wave holds RB 16-row blocks x TW tables.
//
// Row norm: each lane sums the squares of its k values in FP32 (one rounding per fused
// multiply-add, at most d/4 + 3 of them); the four k groups are added in FP32 (two more).
// The sum is scaled by norm_up = 1 + (DP + 2) 2^-23 >= 1 + gamma_{d/4+5}(2^-24), and
// (d + 16) 2^-125 is added for squares lost below the normal range: an upper bound of
// ||x||^2.
template <int TW, int RB, int REM, int KS>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(DIRECT_WAVES, DIRECT_WAVES))) void hash_fp32_direct_kernel(
    const HashArgs a, int64_t tiles_m, int64_t n_slots) {
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);  // wave-uniform: buffer views in SGPRs
    // KS == 1: the waves split the workgroup tile 2 (rows) x 2 (columns).  KS == 4: all four
    // waves take the same 16 RB x 16 TW tile and a quarter of k each (kw).
    const int wm = KS == 1 ? wave >> 1 : 0, wn = KS == 1 ? wave & 1 : 0, kw = KS == 1 ? 0 : wave;
    const int64_t nv = a.n_dev ? *a.n_dev : a.n;
    const int cl = lane & 15, kin = lane >> 4;
    const int d = a.d;
    const uint32_t xo = (uint32_t)(cl * d) * 4u, wo = (uint32_t)(cl * a.DP) * 4u;
    const int xstep = 16 * d * 4, wstep = 16 * a.DP * 4;  // bytes per 16-row / 16-column tile
    // Scalar offsets of the row blocks and column tiles.  readfirstlane keeps each one a
    // scalar operand: a uniform value that reaches a load through a phi the compiler places
    // in a vector register would otherwise get a loop around the load.
    auto xoff = [&](int b) { return __builtin_amdgcn_readfirstlane(b * xstep); };
    auto woff = [&](int t) { return __builtin_amdgcn_readfirstlane(t * wstep); };
    const int nfull = d >> 4;  // full 16-wide k blocks; REM = d - 16 nfull (0, 4, 8 or 12)
    const int kb0 = nfull * kw / KS, kb1 = nfull * (kw + 1) / KS;  // this wave's full blocks
    const float gx = KS == 1 ? a.gx : a.gx_split;

    // Tile slot -> this wave's first row and first padded column; false if it has no rows.
    auto slot_tile = [&](int64_t v, int64_t& rbase, int& cbase) -> bool {
        constexpr int TR = KS == 1 ? 32 * RB : 16 * RB, TC = KS == 1 ? 32 * TW : 16 * TW;
        const int64_t ntn = KS == 1 ? a.n_tiles_n : 2 * a.n_tiles_n;
        const int64_t xcd = v & 7, local = v >> 3;
        const int64_t tile_n = local % ntn;
        const int64_t tile_m = (local / ntn) * 8 + xcd;
        rbase = tile_m * TR + wm * (16 * RB);
        cbase = (int)tile_n * TC + wn * TW * 16;
        return tile_m < tiles_m && rbase < a.n;
    };
    // Range-checked buffer views: the wave's rows of X (rows past n read as zero) and its
    // 16 TW padded columns of W^T.  A lane's offset names its row (column) and k group;
    // the tile index goes into the wave-uniform scalar offset.
    auto x_view = [&](int64_t rbase) {
        const int64_t rows_here = min((int64_t)(16 * RB), a.n - rbase);
        return __builtin_amdgcn_make_buffer_rsrc((void*)(a.X + rbase * (int64_t)d), (short)0,
                                                 (int)(rows_here * d * 4), 0x00020000);
    };
    auto w_view = [&](int cbase) {
        return __builtin_amdgcn_make_buffer_rsrc((void*)(a.Wt + (int64_t)cbase * a.DP), (short)0,
                                                 16 * TW * a.DP * 4, 0x00020000);
    };

    int64_t v = blockIdx.x, rbase = 0;
    int cbase = 0;
    while (v < n_slots && !slot_tile(v, rbase, cbase)) v += gridDim.x;
    if (v >= n_slots) return;
    __amdgpu_buffer_rsrc_t xs = x_view(rbase), ws = w_view(cbase);

    f4 acc[RB][TW];
    float ss[RB];
    auto load_a = [&](int kb, f4 (&av)[RB]) {
        const uint32_t kof = (uint32_t)(kb + 4 * kin) * 4u;
#pragma unroll
        for (int b = 0; b < RB; ++b)
            av[b] = __builtin_bit_cast(f4, __builtin_amdgcn_raw_buffer_load_b128(xs, xo + kof, xoff(b), 0));
    };
    auto load_b = [&](int kb, f4 (&bv)[TW]) {
        const uint32_t kof = (uint32_t)(kb + 4 * kin) * 4u;
#pragma unroll
        for (int t = 0; t < TW; ++t)
            bv[t] = __builtin_bit_cast(f4, __builtin_amdgcn_raw_buffer_load_b128(ws, wo + kof, woff(t), 0));
    };
    auto load = [&](int kb, f4 (&av)[RB], f4 (&bv)[TW]) {
        load_a(kb, av);
        load_b(kb, bv);
    };
    // FIRST: the tile's first k block, whose products start the accumulators (a zero
    // accumulator operand instead of clearing 16 RB TW registers).
    auto step = [&](const f4 (&av)[RB], const f4 (&bv)[TW], auto first) {
        constexpr bool FIRST = decltype(first)::value;
#pragma unroll
        for (int b = 0; b < RB; ++b)
#pragma unroll
            for (int q = 0; q < 4; ++q) ss[b] = fmaf(av[b][q], av[b][q], ss[b]);
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
            for (int t = 0; t < TW; ++t)
#pragma unroll
                for (int b = 0; b < RB; ++b)
                    acc[b][t] = __builtin_amdgcn_mfma_f32_16x16x4f32(
                        av[b][q], bv[t][q], (FIRST && q == 0) ? f4{0.f, 0.f, 0.f, 0.f} : acc[b][t], 0, 0, 0);
    };
    const std::false_type more_k{};

    f4 ac[RB], bc[TW];
    if (kb1 > kb0) load_a(16 * kb0, ac);
    for (;;) {
        if (kb1 > kb0) load_b(16 * kb0, bc);
#pragma unroll
        for (int b = 0; b < RB; ++b) ss[b] = 0.f;
        // Block i + 1 is loaded while block i is multiplied; two blocks per trip so that the
        // operand registers alternate without copies.  Past the last full block the loads
        // read the partial block or the next rows and columns: in range, and unused unless
        // REM == 12, whose partial block it is.
        auto pair = [&](int i, auto first) {
            f4 an[RB], bn[TW];
            load(16 * (i + 1), an, bn);
            step(ac, bc, first);
            // Keep each block's norm updates (which wait for its loads) out of the previous
            // block's MFMA stream.
            __builtin_amdgcn_sched_barrier(0);
            load(16 * (i + 2), ac, bc);
            step(an, bn, more_k);
            __builtin_amdgcn_sched_barrier(0);
        };
        auto single = [&](int i, auto first) {
            f4 an[RB], bn[TW];
            load(16 * (i + 1), an, bn);
            step(ac, bc, first);
            if constexpr (REM == 12) {
#pragma unroll
                for (int b = 0; b < RB; ++b) ac[b] = an[b];
#pragma unroll
                for (int t = 0; t < TW; ++t) bc[t] = bn[t];
            }
        };
        if (kb1 - kb0 >= 2) {
            pair(kb0, std::true_type{});
            int i = kb0 + 2;
            for (; i + 2 <= kb1; i += 2) pair(i, more_k);
            if (i < kb1) single(i, more_k);
        } else if (kb1 > kb0) {
            single(kb0, std::true_type{});
        } else {
#pragma unroll
            for (int b = 0; b < RB; ++b)
#pragma unroll
                for (int t = 0; t < TW; ++t) acc[b][t] = f4{0.f, 0.f, 0.f, 0.f};
        }

        // The partial block belongs to the last k quarter; the other quarters multiply
        // zeros there (adding an exact zero leaves the accumulator unchanged).
        const int kb = 16 * nfull;
        const bool tail_zero = kw != KS - 1;
        if constexpr (REM == 12) {
            if (kb1 == kb0) load(kb, ac, bc);
            if (kin == 3 || tail_zero) {
#pragma unroll
                for (int b = 0; b < RB; ++b) ac[b] = f4{0.f, 0.f, 0.f, 0.f};
            }
            step(ac, bc, more_k);
        } else if constexpr (REM == 8) {
            typedef float f2 __attribute__((ext_vector_type(2)));
            const uint32_t kof = (uint32_t)(kb + 2 * kin) * 4u;
            f2 av[RB], bv[TW];
#pragma unroll
            for (int b = 0; b < RB; ++b) {
                av[b] = __builtin_bit_cast(f2, __builtin_amdgcn_raw_buffer_load_b64(xs, xo + kof, xoff(b), 0));
                if (tail_zero) av[b] = f2{0.f, 0.f};
            }
#pragma unroll
            for (int t = 0; t < TW; ++t)
                bv[t] = __builtin_bit_cast(f2, __builtin_amdgcn_raw_buffer_load_b64(ws, wo + kof, woff(t), 0));
#pragma unroll
            for (int b = 0; b < RB; ++b) ss[b] = fmaf(av[b][1], av[b][1], fmaf(av[b][0], av[b][0], ss[b]));
#pragma unroll
            for (int q = 0; q < 2; ++q)
#pragma unroll
                for (int t = 0; t < TW; ++t)
#pragma unroll
                    for (int b = 0; b < RB; ++b)
                        acc[b][t] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[b][q], bv[t][q], acc[b][t], 0, 0, 0);
        } else if constexpr (REM == 4) {
            const uint32_t kof = (uint32_t)(kb + kin) * 4u;
            float av[RB], bv[TW];
#pragma unroll
            for (int b = 0; b < RB; ++b) {
                av[b] = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(xs, xo + kof, xoff(b), 0));
                if (tail_zero) av[b] = 0.f;
            }
#pragma unroll
            for (int t = 0; t < TW; ++t)
                bv[t] = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(ws, wo + kof, woff(t), 0));
#pragma unroll
            for (int b = 0; b < RB; ++b) ss[b] = fmaf(av[b], av[b], ss[b]);
#pragma unroll
            for (int t = 0; t < TW; ++t)
#pragma unroll
                for (int b = 0; b < RB; ++b)
                    acc[b][t] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[b], bv[t], acc[b][t], 0, 0, 0);
        }

        // This tile's column factors, loaded before the next tile's rows: memory waits
        // count loads in issue order, so the epilogue's wait for these would otherwise also
        // wait for the rows.
        float wcol[TW];
#pragma unroll
        for (int t = 0; t < TW; ++t) wcol[t] = a.wb[cbase + 16 * t + cl];

        // The next tile of this wave; the rows of its first k block are in flight during
        // the epilogue (the W^T block, an L2 hit, is loaded after it).
        int64_t v2 = v + gridDim.x, rbase2 = 0;
        int cbase2 = 0;
        while (v2 < n_slots && !slot_tile(v2, rbase2, cbase2)) v2 += gridDim.x;
        const bool more = v2 < n_slots;
        if (more) {
            xs = x_view(rbase2);
            ws = w_view(cbase2);
            if (kb1 > kb0) load_a(16 * kb0, ac);
        }

        uint32_t tmask = ~0u;
        if constexpr (KS == 4) {
            // Table t of the tile is finished by wave t % 4.  The other three waves hand it
            // their partial sums through LDS; it adds the four as (q0 + q1) + (q2 + q3), in
            // k order whichever wave it is.  Every wave needs the whole row norm.  The first
            // barrier keeps the previous tile's partials until they have been read.
            __shared__ f4 part[TW][3][RB][64];
            __shared__ f4 spart[4][64];
            __syncthreads();
#pragma unroll
            for (int t = 0; t < TW; ++t) {
                const int o = t & 3;
                if (o != kw) {
                    const int sl = kw - (kw > o ? 1 : 0);
#pragma unroll
                    for (int b = 0; b < RB; ++b) part[t][sl][b][lane] = acc[b][t];
                }
            }
            {
                f4 sv = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
                for (int b = 0; b < RB; ++b) sv[b] = ss[b];
                spart[kw][lane] = sv;
            }
            __syncthreads();
            tmask = 0u;
#pragma unroll
            for (int t = 0; t < TW; ++t) {
                if ((t & 3) != kw) continue;
                tmask |= 1u << t;
#pragma unroll
                for (int b = 0; b < RB; ++b) {
                    f4 q[4];
#pragma unroll
                    for (int w = 0; w < 4; ++w) q[w] = (w == kw) ? acc[b][t] : part[t][w - (w > kw ? 1 : 0)][b][lane];
                    acc[b][t] = (q[0] + q[1]) + (q[2] + q[3]);
                    __builtin_amdgcn_sched_barrier(0);  // one tile at a time: few registers in flight
                }
            }
            const f4 s0 = spart[0][lane], s1 = spart[1][lane], s2 = spart[2][lane], s3 = spart[3][lane];
#pragma unroll
            for (int b = 0; b < RB; ++b) ss[b] = (s0[b] + s1[b]) + (s2[b] + s3[b]);
        }
        // Row bound factor gx * ||x||, rounded up by a relative 2^-20; lane cl holds it for
        // row 16b + cl, lane l needs rows 16b + 4 kin + r.  The four k groups' sums are added
        // in FP32 (two more roundings: d/4 + 5 in all, well inside norm_up), then the scaled
        // sum (one rounding), the hardware square root (within one ulp) and two products: at
        // most 5 2^-24 relative below the exact value, covered by the 2^-20 margin.  The
        // (d + 16) 2^-125 term keeps the root's argument a normal number.
        // All row blocks go through each step together (the shuffles' latencies overlap).
        float s2[RB], rbnd[4 * RB];
#pragma unroll
        for (int b = 0; b < RB; ++b) s2[b] = ss[b] + __shfl_xor(ss[b], 16, 64);
#pragma unroll
        for (int b = 0; b < RB; ++b) s2[b] += __shfl_xor(s2[b], 32, 64);
#pragma unroll
        for (int b = 0; b < RB; ++b)
            s2[b] = gx * __builtin_amdgcn_sqrtf(fmaf(s2[b], a.norm_up, (float)(d + 16) * 0x1p-125f)) * (1.f + 0x1p-20f);
#pragma unroll
        for (int b = 0; b < RB; ++b)
#pragma unroll
            for (int r = 0; r < 4; ++r) rbnd[4 * b + r] = __shfl(s2[b], 4 * kin + r, 64);
        sign_epilogue<TW, RB>(a, acc, rbnd, wcol, rbase, cbase, nv, lane, tmask);
        if (!more) break;
        v = v2;
        rbase = rbase2;
        cbase = cbase2;
    }
}

template <int TW>
hipError_t launch_tw(const HashArgs& a, bool vec, hipStream_t s) {
    const int64_t groups = (a.n_tiles_m + 7) / 8;
    const int64_t blocks = groups * 8 * a.n_tiles_n;
    // The direct kernel addresses a wave's 64 rows and 16 TW columns with 32-bit byte offsets;
    // at TW = 8 its accumulators and two operand blocks would not fit in 256 registers.
    if constexpr (TW <= 5) {
        if (vec && (int64_t)a.d * 64 * 4 < ((int64_t)1 << 31) && (int64_t)a.DP * 16 * TW * 4 < ((int64_t)1 << 31)) {
            constexpr int RB = DIRECT_RB;
            const dim3 b(256);
            // Two resident workgroups per CU, rounded up to a multiple of the 8 XCDs.
            const int64_t persist = ((int64_t)cu_count() * DIRECT_WAVES + 7) / 8 * 8;
            if ((a.d >> 4) >= SPLIT_K_BLOCKS) {
                // Long rows: workgroups of 4 waves over 16 RB rows x 16 TW columns, k split
                // four ways (a quarter of the accumulation chain per wave: a 4x tighter bound).
                const int64_t tiles_m = (a.n + 16 * RB - 1) / (16 * RB);
                const int64_t slots = (tiles_m + 7) / 8 * 8 * (2 * a.n_tiles_n);
                const dim3 g((unsigned)(slots < persist ? slots : persist));
                switch (a.d & 15) {
                    case 0: hipLaunchKernelGGL((hash_fp32_direct_kernel<TW, RB, 0, 4>), g, b, 0, s, a, tiles_m, slots); break;
                    case 4: hipLaunchKernelGGL((hash_fp32_direct_kernel<TW, RB, 4, 4>), g, b, 0, s, a, tiles_m, slots); break;
                    case 8: hipLaunchKernelGGL((hash_fp32_direct_kernel<TW, RB, 8, 4>), g, b, 0, s, a, tiles_m, slots); break;
                    default: hipLaunchKernelGGL((hash_fp32_direct_kernel<TW, RB, 12, 4>), g, b, 0, s, a, tiles_m, slots); break;
                }
                return hipGetLastError();
            }
            // Workgroups of 4 waves over 32 RB rows x 32 TW columns.
            const int64_t tiles_m = (a.n + 32 * RB - 1) / (32 * RB);
            const int64_t slots = (tiles_m + 7) / 8 * 8 * a.n_tiles_n;
            const dim3 g((unsigned)(slots < persist ? slots : persist));
            switch (a.d & 15) {
                case 0: hipLaunchKernelGGL((hash_fp32_direct_kernel<TW, RB, 0, 1>), g, b, 0, s, a, tiles_m, slots); break;
                case 4: hipLaunchKernelGGL((hash_fp32_direct_kernel<TW, RB, 4, 1>), g, b, 0, s, a, tiles_m, slots); break;
                case 8: hipLaunchKernelGGL((hash_fp32_direct_kernel<TW, RB, 8, 1>), g, b, 0, s, a, tiles_m, slots); break;
                default: hipLaunchKernelGGL((hash_fp32_direct_kernel<TW, RB, 12, 1>), g, b, 0, s, a, tiles_m, slots); break;
            }
            return hipGetLastError();
        }
    }
    if (vec)
        hipLaunchKernelGGL((hash_fp32_kernel<TW, true>), dim3((unsigned)blocks), dim3(256), 0, s, a);
    else
        hipLaunchKernelGGL((hash_fp32_kernel<TW, false>), dim3((unsigned)blocks), dim3(256), 0, s, a);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_hash_fp32(const HashArgs& a, int TW, bool vec, hipStream_t s) {
    switch (TW) {
        case 1: return launch_tw<1>(a, vec, s);
        case 2: return launch_tw<2>(a, vec, s);
        case 4: return launch_tw<4>(a, vec, s);
        case 5: return launch_tw<5>(a, vec, s);
        case 8: return launch_tw<8>(a, vec, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace ace
