// Internal declarations shared by the host API and the kernels of the ACE library.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/ace.h"

namespace ace {

typedef unsigned long long u64;
typedef unsigned __int128 u128;
typedef __int128 i128;

// Columns per table in the padded projection layout: every table owns 16
// consecutive columns (bits k >= K are zero columns), so one 16-wide MFMA
// output tile is exactly one table.
constexpr int KPAD = 16;
// Contraction padding of the device copy of W.
constexpr int DPAD = 32;
// FP32 rows with at least this many 16-wide k blocks are hashed with the k range split four
// ways over the waves of a workgroup: each accumulation chain is a quarter as long, and so
// is the error bound (fewer projections to refine).
constexpr int SPLIT_K_BLOCKS = 128;

// Arguments of the projection + sign-pack kernels (one per precision).
// Low-precision operands (split-BF16 x_h, x_l, w_h, w_l; e4m3 x^, w^) are stored in
// tiles of 16 rows (or padded columns) so that one 16-row MFMA operand block of a k-step
// is one contiguous read.  Inside a tile a row has 64-byte segments of four 16-byte
// chunks, and chunk c of row r sits at position c ^ tile_chunk_swz(r): fragment reads of
// 16 rows x one chunk out of LDS then hit no bank twice on gfx950.
//   BF16: 16 rows x 32 k (1 KB) per tile, tiles row-major over (row / 16, k / 32).
//   e4m3: 16 rows x 128 k (2 KB) per tile, over (row / 16, k / 128); bytes 64 h .. 64 h + 63
//         of each row form sub-tile h (1 KB).
__host__ __device__ inline int tile_chunk_swz(int r) { return (r >> 1) & 3; }
__host__ __device__ inline size_t bf16_tiled_index(int64_t r, int k, int DP) {
    return ((size_t)(r >> 4) * (size_t)(DP >> 5) + (size_t)(k >> 5)) * 512 + (size_t)(r & 15) * 32 +
           (size_t)((((k & 31) >> 3) ^ tile_chunk_swz((int)(r & 15))) << 3) + (size_t)(k & 7);
}
__host__ __device__ inline size_t fp8_tiled_index(int64_t r, int k, int DP) {
    return ((size_t)(r >> 4) * (size_t)(DP >> 7) + (size_t)(k >> 7)) * 2048 + (size_t)((k >> 6) & 1) * 1024 +
           (size_t)(r & 15) * 64 + (size_t)((((k & 63) >> 4) ^ tile_chunk_swz((int)(r & 15))) << 4) +
           (size_t)(k & 15);
}

struct HashArgs {
    const float* X;        // [n][d] FP32, caller's device memory
    int64_t n;
    int32_t d;
    const float* Wt;       // [NP][DP] FP32: padded column cp = j*16 + k holds w_{jK+k}
    int32_t DP;
    const float* wb;       // [NP] column bound factor (norm of w, rounded up); < 0 for pad columns
    int32_t L, K;
    int32_t n_tiles_n;     // column tiles (each 32*TW padded columns)
    int64_t n_tiles_m;     // row tiles
    float gx;              // row bound factor: gamma * safety
    float gx_split;        // the same for the four-way split-k FP32 kernel (d >= 16 SPLIT_K_BLOCKS)
    float eps_abs;         // absolute term for flushed subnormals
    int32_t refine;
    uint16_t* codes;       // [L][ldc]: code of row i of this chunk in table j at j*ldc + i
    int64_t ldc;
    u64* list;             // queue of uncertain projections: row | column << 32 | raw bit << 63
    u64* list_count;       // entries appended (may exceed list_cap)
    u64 list_cap;
    u64* counters;         // [0] bits refined, [1] refined bits that flipped (queue-full path),
                           // [2] bits inside the bound left unrefined (refine = 2)
    uint16_t* refined;     // [L][ldc] or null: bits decided in place (queue full) are marked
    // Split-BF16 operands and bound factors (BF16 kernel only)
    const uint16_t* Wh;    // [NP][DP] bf16 bits of w_h, in 16 x 32 tiles (bf16_tiled_index)
    const uint16_t* Wl;    // [NP][DP] bf16 bits of w_l, likewise
    const float* wbA;      // [NP] column factors of ||x_h||, ||x_l||, ||rho_x|| and the absolute term;
    const float* wbB;      //      wbA < 0 marks a pad column
    const float* wbC;
    const float* wbE;
    float norm_up;         // rounding-up factor of FP32 sums of squares over d terms
    const uint16_t* Xh;    // [n16][DP] bf16 bits of x_h (convert pass), 16 x 32 tiles, n16 = n rounded up to 16
    const uint16_t* Xl;    // [n16][DP] bf16 bits of x_l, likewise
    const float* rowA;     // [n] ||x_h||, ||x_l||, ||rho_x||, rounded up
    const float* rowB;
    const float* rowC;
    const uint8_t* Xq;     // [n16][DP] e4m3 codes of the scaled rows (FP8 kernel), 16 x 128 tiles
    const uint8_t* Wq;     // [NP][DP] e4m3 codes of the scaled columns, likewise
    // Structured projection (hash_struct kernel): the bound is gx * ||x|| + eps_abs
    const uint32_t* sgn;   // [nblk][3][dp / 32] sign bits of D1, D2, D3 (1 = negate)
    const u64* sgn_lane;   // [nblk][3][64]: bit r of word lane = sign bit of element 64 r + lane
    int32_t dp;            // transform size, a power of two in 64 .. 4096
    int32_t nblk;          // blocks of dp outputs
    int32_t rows_per_wave;
    // Rows that are real (the rest of the n rows are masked out: no codes, no refinement);
    // null means all n.  Lets one captured graph serve every batch of up to n rows.
    const int64_t* n_dev;
};

// Arguments of the FP64 pass over the queued projections.
struct RefineArgs {
    const float* X;
    int32_t d;
    const float* Wt;
    int32_t DP;
    int32_t L, K;
    uint16_t* codes;       // [L][ldc], patched in place
    int64_t ldc;
    uint16_t* refined;     // same layout or null: refined bits are set
    const u64* list;
    const u64* list_count;
    u64 list_cap;
    u64* counters;         // [0] bits refined, [1] refined bits that flipped
    u64* clear_next = nullptr;  // if set, zeroed: the queue counter of the next projection launch
};

// Mark bit cp (padded column) of row `row` in the refined mask, if one was asked for
// (used where a projection epilogue decides a bit itself because the queue is full).
__device__ inline void mark_refined(const HashArgs& a, int64_t row, int cp) {
    const int table = cp >> 4, k = cp & 15;
    if (!a.refined || table >= a.L || k >= a.K) return;
    const uintptr_t ra = reinterpret_cast<uintptr_t>(a.refined + (size_t)table * a.ldc + row);
    atomicOr(reinterpret_cast<uint32_t*>(ra & ~(uintptr_t)3), 1u << (k + ((ra & 2) ? 16 : 0)));
}

// Device-side threshold result (mirrors ace_thresh).
struct DevThresh {
    int64_t n, m_scored;
    double mu, mu_scored, sigma, sigma_table, tau;
    int32_t mode, status;
    uint32_t err;          // the context's error word 0 (a count went below zero) at the launch
    uint32_t pad;
};

// Launchers (enqueue only; return the launch error).
hipError_t launch_hash_fp32(const HashArgs& a, int TW, bool vec, hipStream_t s);
hipError_t launch_convert_bf16(const float* X, int64_t n, int d, int DP, bool vec, uint16_t* Xh, uint16_t* Xl,
                               float* rowA, float* rowB, float* rowC, float norm_up, hipStream_t s);
hipError_t launch_hash_bf16(const HashArgs& a, int TW, hipStream_t s);
hipError_t launch_convert_fp8(const float* X, int64_t n, int d, int DP, bool vec, uint8_t* Xq, float* rowA,
                              float* rowB, float norm_up, hipStream_t s);
hipError_t launch_hash_fp8(const HashArgs& a, int TW, hipStream_t s);
hipError_t launch_refine(const RefineArgs& a, int64_t max_entries, bool vec, hipStream_t s);
// Compute units of the current device (cached per device; 256 if it cannot be read).
int cu_count();
hipError_t launch_hash_struct(const HashArgs& a, hipStream_t s);
hipError_t init_struct_attributes();
// sign = +1 insert, -1 delete
// counts: int32 [L][2^K] (counter_bits 32) or uint16 [L][2^K] (counter_bits 16, saturating;
// dropped increments are added to *drops).
hipError_t launch_count_update(const uint16_t* codes, int64_t ldc, int64_t n, int K, int L, int sign,
                               void* counts, int counter_bits, u64* S2, u64* S3, unsigned* err, u64* drops,
                               hipStream_t s);
// mpart (may be null): room for mpart_cap per-block moment entries (3 u64 each); a launch
// of more than 64 blocks that fits writes them there and adds them to mom in one more block.
hipError_t launch_score(const uint16_t* codes, int64_t ldc, int64_t n, int K, int L, const void* counts,
                        int counter_bits, float* s_out, uint32_t* T_out, u64* mom, hipStream_t s,
                        u64* mpart = nullptr, int64_t mpart_cap = 0);
// out may be host memory mapped for the device (the result then needs no copy).  lim (may
// be null, device memory) receives L tau, the flag limit on T (NaN if the mode's set is empty).
hipError_t launch_threshold(int64_t n, int L, const u64* S2, const u64* S3, const u64* mom, const unsigned* err,
                            int mode, double alpha, DevThresh* out, hipStream_t s, double* lim = nullptr);
hipError_t launch_flags(const uint32_t* T, int64_t n, int L, double tau, int mode, uint8_t* flags, hipStream_t s);
// The same with the limit L tau read from device memory (written by launch_threshold).
hipError_t launch_flags_dev(const uint32_t* T, int64_t n, const double* lim, int mode, uint8_t* flags, hipStream_t s);
hipError_t launch_table_sums(const void* counts, int counter_bits, int K, int L, u64* S2, u64* S3, hipStream_t s);
hipError_t launch_zero(void* p, size_t bytes, hipStream_t s);
// Zero up to four small ranges of 64-bit words (each < 2^31 words; a null pointer with 0
// words is skipped) in one launch.
hipError_t launch_zero_small(u64* p0, int64_t w0, u64* p1, int64_t w1, u64* p2, int64_t w2, u64* p3, int64_t w3,
                             hipStream_t s);
// launch_zero of p (bytes a multiple of 4) and launch_zero_small of the four ranges, in one launch.
hipError_t launch_zero_with_small(void* p, size_t bytes, u64* p0, int64_t w0, u64* p1, int64_t w1, u64* p2,
                                  int64_t w2, u64* p3, int64_t w3, hipStream_t s);
// S[q] = sum_x p(q, x)^K (and S2[q] = sum_x p(q, x)^{2K} when S2 != nullptr); m >= 1.
hipError_t launch_exact_score(const float* Q, int64_t m, const float* X, int64_t n, int d, int K, double* S,
                              double* S2, hipStream_t s);
hipError_t init_kernel_attributes();

}  // namespace ace
