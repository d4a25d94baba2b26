// Context and workspace of the ACE library (host side, shared by the API and the
// serving loop).
#pragma once

#include <vector>

#include "ace_internal.h"

namespace ace {

// Device buffers one hash pipeline needs for a chunk of up to `rows` rows.  Each
// stream that runs the pipeline concurrently owns one.
struct Workspace {
    int64_t rows = 0;
    uint16_t* codes = nullptr;     // [L][rows] (+ 2 elements of padding for the 32-bit patch atomics)
    uint16_t* refined = nullptr;   // same shape, allocated on first request
    u64* list = nullptr;           // queue of uncertain projections
    u64* list_count = nullptr;     // [2]: see cur
    int cur = -1;                  // -1: list_count[0] is cleared by a launch before each projection;
                                   // 0 / 1: the counter the next projection uses, the other one
                                   // being cleared by the FP64 pass of the one before (refine = 1)
    u64 list_alloc = 0;
    uint16_t* xh = nullptr;        // [rows][DP] split-BF16 rows (BF16 precision)
    uint16_t* xl = nullptr;
    uint8_t* xq = nullptr;         // [rows][DP] e4m3 rows (FP8 precision)
    float* rown = nullptr;         // [3][rows] row norms (BF16 / FP8)
};

}  // namespace ace

struct ace_ctx_s {
    ace_config cfg;
    int TW = 5;            // tables per wave in the projection kernel
    int n_tiles_n = 1;     // column tiles
    int NP = 0;            // padded columns allocated (n_tiles_n * 32 * TW)
    int DP = 0;            // padded contraction length
    float gx = 0.f, eps_abs = 0.f;
    float gx_split = 0.f;                     // bound factor of the split-k FP32 kernel

    float* Wt = nullptr;   // [NP][DP]
    float* wb = nullptr;   // [NP]
    uint8_t* Wq = nullptr;   // [NP][DP] e4m3 codes of the scaled columns (FP8 precision)
    uint16_t* Wh = nullptr;  // [NP][DP] split-BF16 hi / lo (BF16 precision)
    uint16_t* Wl = nullptr;
    float* wbA = nullptr;    // [4][NP] BF16 bound factors (A, B, C, absolute)
    uint32_t* sgn = nullptr; // structured projection: sign bits [nblk][3][dp / 32] (null: dense W)
    ace::u64* sgn_lane = nullptr;   // the same bits lane-major: [nblk][3][64], bit r = element 64 r + lane
    int dp = 0, nblk = 0;    // structured transform size and blocks
    float gx_struct = 0.f, eps_struct = 0.f;   // structured bound: gx_struct * |x| + eps_struct
    void* counts = nullptr;      // [L][2^K]: int32, or uint16 with 16-bit counters
    int cbits = 32;              // counter width (32 or 16)
    ace::u64* S2 = nullptr;           // [L]
    ace::u64* S3 = nullptr;           // [L][2]
    ace::u64* mom = nullptr;          // m, sum T, sum T^2 lo, hi
    ace::u64* mpart = nullptr;        // [mpart_cap][3] per-block moments of one score launch
    int64_t mpart_cap = 0;
    ace::u64* rcnt = nullptr;         // bits refined, bits flipped, bits inside the bound left unrefined,
                                      // increments dropped by saturated 16-bit counters
    unsigned* err = nullptr;     // device error flags (1 = a count went below zero)
    ace::DevThresh* thr = nullptr;      // pinned host memory the threshold kernel writes
    ace::DevThresh* thr_dev = nullptr;  // its device address
    double* lim = nullptr;              // L tau of the last threshold, for ace_threshold_flag
    ace::Workspace ws;             // workspace of the stream-ordered calls
    int64_t ws_rows = 0;           // rows per internal chunk
    ace::u64 list_cap = 0;              // queue entries used per chunk (<= allocated)

    int64_t n_total = 0;
    int64_t cap = INT32_MAX;
    ace::u64 bits_hashed = 0;
    size_t bytes = 0;
    ace_status sticky = ACE_OK;
    int fail_next = 0;
    int server_attached = 0;       // a serving loop owns the context (ace_destroy refused)

    // Event timing: pairs of (start, end, class) recorded while profiling is on.
    int profiling = 0;
    struct Timed { hipEvent_t a, b; int cls; int64_t rows; };
    std::vector<Timed> timed;
    std::vector<hipEvent_t> pool;
};


namespace ace {

ace_status dev_alloc(ace_ctx c, void** p, size_t bytes);
ace_status ws_alloc(ace_ctx c, Workspace* w, int64_t rows);
void ws_free(Workspace* w);
ace_status check(ace_ctx c, hipError_t e);
// Hash rows [0, n) of X into w->codes [L][n] (projection + sign-pack, then the FP64
// pass over the queued projections when refine = 1).  n_dev (may be null): device count of
// the real rows (<= n); rows beyond it get no codes and no refinement, so a graph captured
// for n rows serves any smaller batch.  count_bits: add n K L to the hashed-bit counter.
ace_status hash_chunk(ace_ctx c, Workspace* w, const float* X, int64_t n, bool want_refined, hipStream_t s,
                      const int64_t* n_dev = nullptr, bool count_bits = true);
// Resolve, once per device, the device address of the static scratch array that
// ace_hash_static uses (the device must be current).
ace_status scratch_bind(int device);

}  // namespace ace
