// Host side of the ACE C ABI: validation, device state, chunking and launches.
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include <cmath>
#include <new>
#include <vector>

#include "ace_context.h"

using namespace ace;

namespace ace {

ace_status dev_alloc(ace_ctx c, void** p, size_t bytes) {
    if (c->cfg.mem_budget > 0 && c->bytes + bytes > (size_t)c->cfg.mem_budget) return ACE_E_NOMEM;
    if (hipMalloc(p, bytes) != hipSuccess) {
        (void)hipGetLastError();
        *p = nullptr;
        return ACE_E_NOMEM;
    }
    c->bytes += bytes;
    return ACE_OK;
}

// Record a launch result: a failed launch makes the context sticky.
ace_status check(ace_ctx c, hipError_t e) {
    if (e != hipSuccess) {
        (void)hipGetLastError();
        c->sticky = ACE_E_DEVICE;
        return ACE_E_DEVICE;
    }
    return ACE_OK;
}

void ws_free(Workspace* w) {
    void* ptrs[] = {w->codes, w->refined, w->list, w->list_count, w->xh, w->xl, w->xq, w->rown};
    for (void* p : ptrs)
        if (p) (void)hipFree(p);
    *w = Workspace();
}

ace_status ws_alloc(ace_ctx c, Workspace* w, int64_t rows) {
    const size_t L = (size_t)c->cfg.L;
    w->rows = rows;
    ace_status st = dev_alloc(c, (void**)&w->codes, sizeof(uint16_t) * (L * rows + 2));
    // Queue for projections inside the bound: 1/32 of a chunk's bits (a full queue only
    // slows the epilogue down, it never changes a result).
    w->list_alloc = (u64)rows * (u64)L * KPAD / 32;
    if (w->list_alloc < 65536) w->list_alloc = 65536;
    st = st ? st : dev_alloc(c, (void**)&w->list, sizeof(u64) * (size_t)w->list_alloc);
    st = st ? st : dev_alloc(c, (void**)&w->list_count, 2 * sizeof(u64));
    if (c->cfg.precision == ACE_BF16) {
        // whole 16-row tiles (the convert pass zeroes the rows past the chunk's last)
        const size_t rows16 = (size_t)(rows + 15) / 16 * 16;
        st = st ? st : dev_alloc(c, (void**)&w->xh, sizeof(uint16_t) * rows16 * c->DP);
        st = st ? st : dev_alloc(c, (void**)&w->xl, sizeof(uint16_t) * rows16 * c->DP);
    }
    if (c->cfg.precision == ACE_FP8E4M3)
        st = st ? st : dev_alloc(c, (void**)&w->xq, (size_t)(rows + 15) / 16 * 16 * c->DP);
    if (c->cfg.precision != ACE_FP32) st = st ? st : dev_alloc(c, (void**)&w->rown, sizeof(float) * 3 * (size_t)rows);
    if (st) ws_free(w);
    return st;
}

}  // namespace ace

namespace {

struct DeviceGuard {
    int prev = -1;
    bool ok = true;
    explicit DeviceGuard(int dev) {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        ok = hipSetDevice(dev) == hipSuccess;
    }
    ~DeviceGuard() {
        if (prev >= 0) (void)hipSetDevice(prev);
    }
};

enum { CLS_HASH = 0, CLS_UPDATE = 1, CLS_SCORE = 2, CLS_OTHER = 3, CLS_REFINE = 4, CLS_CONVERT = 5 };

hipEvent_t take_event(ace_ctx c) {
    if (!c->pool.empty()) {
        hipEvent_t e = c->pool.back();
        c->pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) {
        (void)hipGetLastError();
        return nullptr;
    }
    return e;
}

// Bracket one launch with events when profiling is on.
struct Bracket {
    ace_ctx c;
    hipStream_t s;
    int cls;
    int64_t rows;
    hipEvent_t a = nullptr;
    Bracket(ace_ctx c_, hipStream_t s_, int cls_, int64_t rows_ = 0) : c(c_), s(s_), cls(cls_), rows(rows_) {
        if (c->profiling) {
            a = take_event(c);
            if (a) (void)hipEventRecord(a, s);
        }
    }
    ~Bracket() {
        if (a) {
            hipEvent_t b = take_event(c);
            if (b && hipEventRecord(b, s) == hipSuccess) c->timed.push_back({a, b, cls, rows});
            else c->pool.push_back(a);
        }
    }
};

void free_all(ace_ctx c) {
    for (auto& t : c->timed) {
        (void)hipEventDestroy(t.a);
        (void)hipEventDestroy(t.b);
    }
    for (auto e : c->pool) (void)hipEventDestroy(e);
    c->timed.clear();
    c->pool.clear();
    void* ptrs[] = {c->Wt,  c->wb,  c->Wq,    c->Wh,   c->Wl,  c->wbA, c->counts,  c->S2, c->S3,
                    c->mom, c->lim, c->mpart, c->rcnt, c->err, c->sgn, c->sgn_lane};
    ws_free(&c->ws);
    for (void* p : ptrs)
        if (p) (void)hipFree(p);
    if (c->thr) (void)hipHostFree(c->thr);
}

ace_status enter(ace_ctx c) {
    if (!c) return ACE_E_INVALID;
    if (c->sticky != ACE_OK) return c->sticky;
    return ACE_OK;
}

// A debug hook turns the next enqueueing call into a device failure.
bool take_injected_failure(ace_ctx c) {
    if (c->fail_next) {
        c->fail_next = 0;
        c->sticky = ACE_E_DEVICE;
        return true;
    }
    return false;
}

// Round-to-nearest-even FP32 -> BF16 (finite inputs), the same rounding the kernels use.
uint16_t host_bf16_bits(float x) {
    uint32_t u;
    memcpy(&u, &x, 4);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
float host_bf16_val(uint16_t h) {
    const uint32_t u = (uint32_t)h << 16;
    float x;
    memcpy(&x, &u, 4);
    return x;
}

// OCP e4m3 encoding (bias 7, max 448) with round-to-nearest-even of |v| <= 448, the same
// rounding the device conversion uses; *q receives the encoded value.
uint8_t host_e4m3(float v, float* q) {
    const float a = fabsf(v);
    const uint8_t s = std::signbit(v) ? 0x80 : 0;
    if (a < 0x1p-6f) {
        const float m = nearbyintf(a * 512.f);
        *q = copysignf(m * 0x1p-9f, v);
        return (uint8_t)(s | (uint8_t)m);
    }
    uint32_t u;
    memcpy(&u, &a, 4);
    u += 0x7FFFFu + ((u >> 20) & 1u);
    u &= 0xFFF00000u;
    float r;
    memcpy(&r, &u, 4);
    *q = copysignf(r, v);
    const uint32_t E = ((u >> 23) & 0xFFu) - 127u + 7u;
    const uint32_t M = (u >> 20) & 7u;
    return (uint8_t)(s | (E << 3) | M);
}

int pick_tw(int L, bool fp32) {
    // The split-BF16 kernel holds two accumulator chains and is built for TW <= 4.  Its
    // time goes to moving operand tiles, so a wider tile pays for a few padded tables:
    // take the widest whose padding is at most L / 16 (connection-log L = 50: TW = 2,
    // 0.54 against 0.63 ms at TW = 1 and 0.56 at TW = 4; heavy-tail L = 100: TW = 4,
    // 9.39 against 9.70 ms per 250k rows at TW = 2).
    if (!fp32) {
        for (int tw : {4, 2}) {
            const long pad = (long)(L + 2 * tw - 1) / (2 * tw) * (2 * tw) - L;
            if (16 * pad <= L) return tw;
        }
        return 1;
    }
    // FP32 and e4m3: fewest padded tables; ties go to the wider tile.  (TW = 8 never wins:
    // its padding is never below that of TW = 4.)
    const int cand[] = {5, 4, 2, 1};
    int best = 5;
    long best_pad = -1;
    for (int tw : cand) {
        const long tiles = (L + 2 * tw - 1) / (2 * tw);
        const long pad = tiles * 2 * tw - L;
        if (best_pad < 0 || pad < best_pad) {
            best_pad = pad;
            best = tw;
        }
    }
    return best;
}

}  // namespace

// Hash rows [0, n) of X (one chunk of at most w->rows rows) into the workspace codes
// [L][n]: projection + sign-pack, then the FP64 pass over the queued projections.
ace_status ace::hash_chunk(ace_ctx c, Workspace* w, const float* X, int64_t n, bool want_refined, hipStream_t s,
                           const int64_t* n_dev, bool count_bits) {
    // The queue counter: cleared here, or (a workspace that alternates two counters, with the
    // FP64 pass on) already cleared by the previous chunk's FP64 pass.
    const bool alt = w->cur >= 0 && c->cfg.refine == 1;
    u64* const cnt = alt ? w->list_count + w->cur : w->list_count;
    ace_status st = ACE_OK;
    if (!alt) {
        st = check(c, launch_zero(w->list_count, sizeof(u64), s));
        if (st) return st;
    }
    if (want_refined) {
        st = check(c, launch_zero(w->refined, sizeof(uint16_t) * ((size_t)c->cfg.L * n + 2), s));
        if (st) return st;
    }
    HashArgs a;
    a.X = X;
    a.n = n;
    a.d = c->cfg.d;
    a.Wt = c->Wt;
    a.DP = c->DP;
    a.wb = c->wb;
    a.L = c->cfg.L;
    a.K = c->cfg.K;
    a.n_tiles_n = c->n_tiles_n;
    a.n_tiles_m = (n + 127) / 128;
    a.gx = c->gx;
    a.gx_split = c->gx_split;
    a.eps_abs = c->eps_abs;
    a.refine = c->cfg.refine;
    a.codes = w->codes;
    a.ldc = n;
    a.list = w->list;
    a.list_count = cnt;
    a.list_cap = c->list_cap < w->list_alloc ? c->list_cap : w->list_alloc;
    a.refined = want_refined ? w->refined : nullptr;
    a.counters = c->rcnt;
    a.Wh = c->Wh;
    a.Wl = c->Wl;
    a.wbA = c->wbA;
    a.wbB = c->wbA ? c->wbA + c->NP : nullptr;
    a.wbC = c->wbA ? c->wbA + 2 * c->NP : nullptr;
    a.wbE = c->wbA ? c->wbA + 3 * c->NP : nullptr;
    a.norm_up = (float)(1.0 + ldexp((double)c->DP + 2.0, -23));
    a.n_dev = n_dev;
    const bool vec = (c->cfg.d % 4 == 0) && ((reinterpret_cast<uintptr_t>(X) & 15u) == 0);
    if (count_bits) c->bits_hashed += (u64)n * (u64)c->cfg.K * (u64)c->cfg.L;
    if (c->cfg.precision == ACE_FP8E4M3) {
        {
            Bracket br(c, s, CLS_CONVERT, n);
            st = check(c, launch_convert_fp8(X, n, c->cfg.d, c->DP, vec, w->xq, w->rown, w->rown + w->rows,
                                             a.norm_up, s));
        }
        if (st) return st;
        a.Xq = w->xq;
        a.Wq = c->Wq;
        a.rowA = w->rown;
        a.rowB = w->rown + w->rows;
        Bracket br(c, s, CLS_HASH, n);
        st = check(c, launch_hash_fp8(a, c->TW, s));
    } else if (c->cfg.precision == ACE_BF16) {
        {
            Bracket br(c, s, CLS_CONVERT, n);
            st = check(c, launch_convert_bf16(X, n, c->cfg.d, c->DP, vec, w->xh, w->xl, w->rown,
                                              w->rown + w->rows, w->rown + 2 * w->rows, a.norm_up, s));
        }
        if (st) return st;
        a.Xh = w->xh;
        a.Xl = w->xl;
        a.rowA = w->rown;
        a.rowB = w->rown + w->rows;
        a.rowC = w->rown + 2 * w->rows;
        Bracket br(c, s, CLS_HASH, n);
        st = check(c, launch_hash_bf16(a, c->TW, s));
    } else if (c->sgn) {
        a.sgn = c->sgn;
        a.sgn_lane = c->sgn_lane;
        a.dp = c->dp;
        a.nblk = c->nblk;
        a.rows_per_wave = 4;
        a.gx = c->gx_struct;
        a.eps_abs = c->eps_struct;
        Bracket br(c, s, CLS_HASH, n);
        st = check(c, launch_hash_struct(a, s));
    } else {
        Bracket br(c, s, CLS_HASH, n);
        st = check(c, launch_hash_fp32(a, c->TW, vec, s));
    }
    if (st || c->cfg.refine != 1) return st;
    RefineArgs r;
    r.X = X;
    r.d = c->cfg.d;
    r.Wt = c->Wt;
    r.DP = c->DP;
    r.L = c->cfg.L;
    r.K = c->cfg.K;
    r.codes = w->codes;
    r.ldc = n;
    r.refined = want_refined ? w->refined : nullptr;
    r.list = w->list;
    r.list_count = cnt;
    r.list_cap = a.list_cap;
    r.counters = c->rcnt;
    r.clear_next = alt ? w->list_count + (w->cur ^ 1) : nullptr;
    Bracket br(c, s, CLS_REFINE, n);
    st = check(c, launch_refine(r, (int64_t)a.list_cap, vec, s));
    if (!st && alt) w->cur ^= 1;
    return st;
}

namespace {

ace_status update_rows(ace_ctx c, const float* X, int64_t n, int sign, hipStream_t s) {
    for (int64_t r0 = 0; r0 < n; r0 += c->ws_rows) {
        const int64_t m = (n - r0 < c->ws_rows) ? n - r0 : c->ws_rows;
        ace_status st = hash_chunk(c, &c->ws, X + r0 * (int64_t)c->cfg.d, m, false, s);
        if (st != ACE_OK) return st;
        {
            Bracket br(c, s, CLS_UPDATE, m);
            st = check(c, launch_count_update(c->ws.codes, m, m, c->cfg.K, c->cfg.L, sign, c->counts, c->cbits, c->S2,
                                              c->S3, c->err, c->rcnt + 3, s));
        }
        if (st != ACE_OK) return st;
    }
    return ACE_OK;
}

}  // namespace

extern "C" {

const char* ace_status_string(ace_status s) {
    switch (s) {
        case ACE_OK: return "ACE_OK";
        case ACE_E_INVALID: return "ACE_E_INVALID";
        case ACE_E_NOMEM: return "ACE_E_NOMEM";
        case ACE_E_OVERFLOW: return "ACE_E_OVERFLOW";
        case ACE_E_EMPTY: return "ACE_E_EMPTY";
        case ACE_E_DEVICE: return "ACE_E_DEVICE";
        case ACE_E_STATE: return "ACE_E_STATE";
        case ACE_E_TIMEOUT: return "ACE_E_TIMEOUT";
        default: return "ACE_E_UNKNOWN";
    }
}

const char* ace_version(void) { return "ace-mi355x 0.1 (gfx950)"; }

namespace {

// Transform size and blocks of the structured projection: dp = max(64, next power of two
// >= d) outputs per block, ceil(K L / dp) blocks.
void structured_shape(int d, int K, int L, int* dp, int* nblk) {
    int p = 64;
    while (p < d) p *= 2;
    *dp = p;
    *nblk = (K * L + p - 1) / p;
}

// Dense equivalent of the structured projection, [d][K L] like a caller's W: row c of
// M_b = H D3 H D2 H D1 is (D1 H D2 H D3 H e_i)^T (H symmetric, D diagonal), computed with an
// exact integer fast Walsh-Hadamard transform.  Entries are integers of magnitude <= dp^2.
void structured_dense(const uint8_t* signs, int d, int K, int L, int dp, std::vector<float>& W) {
    const int KL = K * L;
    W.assign((size_t)d * KL, 0.f);
    std::vector<int64_t> v(dp);
    auto fwht = [&]() {
        for (int h = 1; h < dp; h <<= 1)
            for (int i = 0; i < dp; i += 2 * h)
                for (int k = i; k < i + h; ++k) {
                    const int64_t a = v[k], b = v[k + h];
                    v[k] = a + b;
                    v[k + h] = a - b;
                }
    };
    for (int c = 0; c < KL; ++c) {
        const int b = c / dp, i = c % dp;
        const uint8_t* s1 = signs + ((size_t)b * 3 + 0) * dp;
        const uint8_t* s2 = s1 + dp;
        const uint8_t* s3 = s2 + dp;
        for (int u = 0; u < dp; ++u) v[u] = (__builtin_popcount((unsigned)(i & u)) & 1) ? -1 : 1;   // H e_i
        for (int u = 0; u < dp; ++u) v[u] = s3[u] ? -v[u] : v[u];
        fwht();
        for (int u = 0; u < dp; ++u) v[u] = s2[u] ? -v[u] : v[u];
        fwht();
        for (int t = 0; t < d; ++t) W[(size_t)t * KL + c] = (float)(s1[t] ? -v[t] : v[t]);
    }
}

ace_status create_impl(const ace_config* cfg, const float* W_host, const uint8_t* signs, ace_ctx* out);

}  // namespace

ace_status ace_create(const ace_config* cfg, const float* W_host, ace_ctx* out) {
    if (!cfg || !W_host || !out) return ACE_E_INVALID;
    return create_impl(cfg, W_host, nullptr, out);
}

ace_status ace_create_structured(const ace_config* cfg, const uint8_t* signs, ace_ctx* out) {
    if (!cfg || !signs || !out) return ACE_E_INVALID;
    if (cfg->precision != ACE_FP32) return ACE_E_INVALID;
    if (cfg->d < 1 || cfg->d > 4096 || cfg->K < 1 || cfg->K > 16 || cfg->L < 1 || cfg->L > 4096) return ACE_E_INVALID;
    int dp, nblk;
    structured_shape(cfg->d, cfg->K, cfg->L, &dp, &nblk);
    for (size_t i = 0; i < (size_t)nblk * 3 * dp; ++i)
        if (signs[i] > 1) return ACE_E_INVALID;
    std::vector<float> W;
    structured_dense(signs, cfg->d, cfg->K, cfg->L, dp, W);
    return create_impl(cfg, W.data(), signs, out);
}

namespace {

ace_status create_impl(const ace_config* cfg, const float* W_host, const uint8_t* signs, ace_ctx* out) {
    if (cfg->d < 1 || cfg->K < 1 || cfg->K > 16 || cfg->L < 1 || cfg->L > 4096) return ACE_E_INVALID;
    if (cfg->precision != ACE_FP32 && cfg->precision != ACE_BF16 && cfg->precision != ACE_FP8E4M3)
        return ACE_E_INVALID;
    if (cfg->refine < 0 || cfg->refine > 2) return ACE_E_INVALID;
    if (cfg->max_batch_rows < 0 || cfg->mem_budget < 0 || cfg->device < 0) return ACE_E_INVALID;
    if (cfg->bound_model != ACE_BOUND_MEASURED && cfg->bound_model != ACE_BOUND_GENERIC) return ACE_E_INVALID;
    // The generic model charges each addition a rounding of 2^-23 relative to the sum; the
    // e4m3 instruction is measured to drop bits far above that (about 2^-13 of a k-group's
    // largest product), so no generic bound is offered for it.
    if (cfg->precision == ACE_FP8E4M3 && cfg->bound_model == ACE_BOUND_GENERIC) return ACE_E_INVALID;
    if (cfg->counter_bits != 0 && cfg->counter_bits != 16 && cfg->counter_bits != 32) return ACE_E_INVALID;
    if ((int64_t)cfg->d > (int64_t)1 << 24) return ACE_E_INVALID;

    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || cfg->device >= ndev) {
        (void)hipGetLastError();
        return ACE_E_DEVICE;
    }
    DeviceGuard g(cfg->device);
    if (!g.ok) return ACE_E_DEVICE;
    static bool attrs_done = false;
    if (!attrs_done) {
        if (init_kernel_attributes() != hipSuccess) {
            (void)hipGetLastError();
            return ACE_E_DEVICE;
        }
        attrs_done = true;
    }
    // The allocation-free entry point's scratch on this device; a failure here is reported
    // by that entry point, which retries the binding.
    (void)scratch_bind(cfg->device);

    ace_ctx c = new (std::nothrow) ace_ctx_s();
    if (!c) return ACE_E_NOMEM;
    c->cfg = *cfg;
    if (c->cfg.max_batch_rows == 0) c->cfg.max_batch_rows = (int64_t)1 << 20;
    const int d = cfg->d, K = cfg->K, L = cfg->L;
    c->TW = pick_tw(L, cfg->precision != ACE_BF16);
    c->n_tiles_n = (L + 2 * c->TW - 1) / (2 * c->TW);
    c->NP = c->n_tiles_n * 32 * c->TW;
    const int dpad = cfg->precision == ACE_FP8E4M3 ? 128 : DPAD;  // FP8 k-steps are 128 wide
    c->DP = (d + dpad - 1) / dpad * dpad;
    // FP32 bound factor gamma_h(u), rounded up by a relative 2^-16 for the FP32 bound product:
    //   measured model: exact products, one round-to-nearest per product added -> h = DP + 4, u = 2^-24
    //   generic model:  up to 6 units of 2^-23 per 4-product instruction        -> h = 2 DP + 8, u = 2^-23
    // The split-k kernel's chains hold at most P = 16 ceil(nfull / 4) + 16 products, and the
    // four partial sums are added in two more roundings: h = P + 6 (measured), 2 P + 10 (generic).
    {
        const bool gen = cfg->bound_model == ACE_BOUND_GENERIC;
        const double u = ldexp(1.0, gen ? -23 : -24);
        const double h = gen ? 2.0 * c->DP + 8.0 : (double)c->DP + 4.0;
        c->gx = (float)(h * u / (1.0 - h * u) * (1.0 + ldexp(1.0, -16)));
        const double P = 16.0 * (double)(((d >> 4) + 3) / 4) + 16.0;
        const double hs = gen ? 2.0 * P + 10.0 : P + 6.0;
        c->gx_split = (float)(hs * u / (1.0 - hs * u) * (1.0 + ldexp(1.0, -16)));
        c->eps_abs = (float)((2.0 * c->DP + 8.0) * ldexp(1.0, -125));
    }
    c->ws_rows = c->cfg.max_batch_rows;

    const int64_t B = (int64_t)1 << K;
    ace_status st = ACE_OK;
    st = st ? st : dev_alloc(c, (void**)&c->Wt, sizeof(float) * (size_t)c->NP * c->DP);
    st = st ? st : dev_alloc(c, (void**)&c->wb, sizeof(float) * (size_t)c->NP);
    if (cfg->precision == ACE_FP8E4M3) {
        st = st ? st : dev_alloc(c, (void**)&c->Wq, (size_t)c->NP * c->DP);
        st = st ? st : dev_alloc(c, (void**)&c->wbA, sizeof(float) * 4 * (size_t)c->NP);
    }
    if (cfg->precision == ACE_BF16) {
        st = st ? st : dev_alloc(c, (void**)&c->Wh, sizeof(uint16_t) * (size_t)c->NP * c->DP);
        st = st ? st : dev_alloc(c, (void**)&c->Wl, sizeof(uint16_t) * (size_t)c->NP * c->DP);
        st = st ? st : dev_alloc(c, (void**)&c->wbA, sizeof(float) * 4 * (size_t)c->NP);
    }
    c->cbits = cfg->counter_bits == 16 ? 16 : 32;
    st = st ? st : dev_alloc(c, (void**)&c->counts, (size_t)(c->cbits / 8) * (size_t)L * B);
    st = st ? st : dev_alloc(c, (void**)&c->S2, sizeof(u64) * (size_t)L);
    st = st ? st : dev_alloc(c, (void**)&c->S3, sizeof(u64) * 2 * (size_t)L);
    st = st ? st : dev_alloc(c, (void**)&c->mom, sizeof(u64) * 4);
    st = st ? st : dev_alloc(c, (void**)&c->lim, sizeof(double));
    // Per-block moments of a score launch over one workspace chunk (either score kernel).
    c->mpart_cap = (c->ws_rows + 255) / 256 + 1;
    st = st ? st : dev_alloc(c, (void**)&c->mpart, sizeof(u64) * 3 * (size_t)c->mpart_cap);
    st = st ? st : dev_alloc(c, (void**)&c->rcnt, sizeof(u64) * 4);
    st = st ? st : dev_alloc(c, (void**)&c->err, sizeof(unsigned) * 4);
    // The threshold result goes straight to coherent pinned host memory: no copy after the
    // kernel, and the stream synchronisation that ends the call makes it visible.
    if (!st && (hipHostMalloc((void**)&c->thr, sizeof(DevThresh), hipHostMallocCoherent) != hipSuccess ||
                hipHostGetDevicePointer((void**)&c->thr_dev, c->thr, 0) != hipSuccess)) {
        (void)hipGetLastError();
        st = ACE_E_NOMEM;
    }
    st = st ? st : ws_alloc(c, &c->ws, c->ws_rows);
    // The context's own workspace alternates its two queue counters (both start at zero).
    if (!st) st = check(c, hipMemset(c->ws.list_count, 0, 2 * sizeof(u64)));
    if (!st) c->ws.cur = 0;
    c->list_cap = c->ws.list_alloc;
    if (signs) {
        structured_shape(d, K, L, &c->dp, &c->nblk);
        // dp / 32 words per diagonal, padded so that 64-bit loads of the last word stay inside
        st = st ? st : dev_alloc(c, (void**)&c->sgn, sizeof(uint32_t) * ((size_t)c->nblk * 3 * (c->dp / 32) + 2));
        st = st ? st : dev_alloc(c, (void**)&c->sgn_lane, sizeof(u64) * (size_t)c->nblk * 3 * 64);
        // Bound of the three FP32 transforms: g dp^1.5 |x| (3 + 4g), g = m u (1 + 2u)^m,
        // u = 2^-24, m = log2 dp (rounded up for the FP32 product with |x|).
        const double u = ldexp(1.0, -24), m = log2((double)c->dp);
        const double gg = m * u * pow(1.0 + 2.0 * u, m);
        c->gx_struct = (float)(gg * pow((double)c->dp, 1.5) * (3.0 + 4.0 * gg) * (1.0 + ldexp(1.0, -16)));
        c->eps_struct = (float)ldexp(1.0, -90);
    }
    if (st != ACE_OK) {
        free_all(c);
        delete c;
        return st;
    }
    // Padded device copy of W: column cp = j*16 + k holds w_{jK+k}; zero elsewhere.
    std::vector<float> Wt((size_t)c->NP * c->DP, 0.f);
    std::vector<float> wb((size_t)c->NP, -1.f);
    for (int j = 0; j < L; ++j)
        for (int k = 0; k < K; ++k) {
            const int cp = j * KPAD + k;
            double ss = 0.0;
            for (int t = 0; t < d; ++t) {
                const float w = W_host[(size_t)t * K * L + (size_t)j * K + k];
                Wt[(size_t)cp * c->DP + t] = w;
                ss += (double)w * (double)w;
            }
            wb[cp] = (float)(sqrt(ss) * (1.0 + ldexp(1.0, -20)));
        }
    hipError_t e = hipSuccess;
    if (cfg->precision == ACE_BF16) {
        // Exact split w = w_h + w_l + rho_w and the column factors of the error bound
        // (see the BF16 kernel): I = DP/32 MFMA instructions per chain, u = 2^-23.
        std::vector<uint16_t> Wh((size_t)c->NP * c->DP, 0), Wl((size_t)c->NP * c->DP, 0);
        std::vector<float> f((size_t)4 * c->NP, 0.f);
        for (int cp = 0; cp < c->NP; ++cp) f[cp] = -1.f;
        const double uu = ldexp(1.0, -23), I = (double)c->DP / 32.0, up = 1.0 + ldexp(1.0, -10);
        // Accumulation error per chain, in units of u = 2^-23 times sum |products|:
        //   generic:  34 per instruction                    -> main 34 I,     corr 68 I
        //   measured: 8 x 2^-24 group truncation once, plus  -> main 4 + 2 I,  corr 4 + 4 I
        //             four roundings of 2^-24 per instruction
        const bool gen = cfg->bound_model == ACE_BOUND_GENERIC;
        const double hm = gen ? 34.0 * I : 4.0 + 2.0 * I;
        const double hc = gen ? 68.0 * I : 4.0 + 4.0 * I;
        for (int j = 0; j < L; ++j)
            for (int k = 0; k < K; ++k) {
                const int cp = j * KPAD + k;
                double nh = 0, nl = 0, nr = 0, nw = 0;
                for (int t = 0; t < d; ++t) {
                    const float w = W_host[(size_t)t * K * L + (size_t)j * K + k];
                    const uint16_t hb = host_bf16_bits(w);
                    const float hv = host_bf16_val(hb);
                    const float r1 = w - hv;
                    const uint16_t lb = host_bf16_bits(r1);
                    const float lv = host_bf16_val(lb);
                    const float r2 = r1 - lv;
                    Wh[bf16_tiled_index(cp, t, c->DP)] = hb;
                    Wl[bf16_tiled_index(cp, t, c->DP)] = lb;
                    nh += (double)hv * hv;
                    nl += (double)lv * lv;
                    nr += (double)r2 * r2;
                    nw += (double)w * w;
                }
                nh = sqrt(nh);
                nl = sqrt(nl);
                nr = sqrt(nr);
                nw = sqrt(nw);
                f[cp] = (float)((nr + hm * uu * nh + hc * uu * nl + 2.0 * uu * (nh + nl)) * up);
                f[c->NP + cp] = (float)((nl + nr + hc * uu * nh + 2.0 * uu * nh) * up);
                f[2 * c->NP + cp] = (float)(nw * up);
                f[3 * c->NP + cp] = (float)(3.0 * ldexp(1.0, -126) * sqrt((double)c->DP) * (nw + 1.0) * up);
            }
        e = hipMemcpy(c->Wh, Wh.data(), Wh.size() * sizeof(uint16_t), hipMemcpyHostToDevice);
        if (e == hipSuccess) e = hipMemcpy(c->Wl, Wl.data(), Wl.size() * sizeof(uint16_t), hipMemcpyHostToDevice);
        if (e == hipSuccess) e = hipMemcpy(c->wbA, f.data(), f.size() * sizeof(float), hipMemcpyHostToDevice);
    }
    if (e == hipSuccess && cfg->precision == ACE_FP8E4M3) {
        // Per-column power-of-two scale s_c (max |w| / s_c <= 448), e4m3 codes of w / s_c,
        // and the column factors of the bound (see the FP8 kernel), in scaled units.
        std::vector<uint8_t> Wq((size_t)c->NP * c->DP, 0);
        std::vector<float> f((size_t)4 * c->NP, 0.f);
        for (int cp = 0; cp < c->NP; ++cp) f[cp] = -1.f;
        const double I = (double)c->DP / 128.0, up = 1.0 + ldexp(1.0, -10);
        const double hacc = ldexp(1.0, -9) + 8.0 * I * ldexp(1.0, -24);
        for (int j = 0; j < L; ++j)
            for (int k = 0; k < K; ++k) {
                const int cp = j * KPAD + k;
                float mx = 0.f;
                for (int t = 0; t < d; ++t) mx = fmaxf(mx, fabsf(W_host[(size_t)t * K * L + (size_t)j * K + k]));
                int ex = 0;
                if (mx > 0.f) {
                    ex = ilogbf(mx / 448.f);
                    while (ldexpf(mx, -ex) > 448.f) ++ex;
                }
                double nq = 0, nd = 0;
                for (int t = 0; t < d; ++t) {
                    const float w = ldexpf(W_host[(size_t)t * K * L + (size_t)j * K + k], -ex);
                    float q;
                    Wq[fp8_tiled_index(cp, t, c->DP)] = host_e4m3(w, &q);
                    nq += (double)q * q;
                    nd += (double)(w - q) * (w - q);
                }
                nq = sqrt(nq);
                nd = sqrt(nd);
                f[cp] = (float)((nd + hacc * nq) * up);
                f[c->NP + cp] = (float)((nq + nd) * up);
                f[3 * c->NP + cp] = (float)((double)c->DP * ldexp(1.0, -140) * (nq + 1.0) * up);
            }
        e = hipMemcpy(c->Wq, Wq.data(), Wq.size(), hipMemcpyHostToDevice);
        if (e == hipSuccess) e = hipMemcpy(c->wbA, f.data(), f.size() * sizeof(float), hipMemcpyHostToDevice);
    }
    if (e == hipSuccess && signs) {
        std::vector<uint32_t> words((size_t)c->nblk * 3 * (c->dp / 32) + 2, 0u);
        std::vector<u64> lanes((size_t)c->nblk * 3 * 64, 0ull);
        for (size_t i = 0; i < (size_t)c->nblk * 3 * c->dp; ++i)
            if (signs[i]) {
                words[i >> 5] |= 1u << (i & 31);
                const size_t diag = i / c->dp, el = i % c->dp;
                lanes[diag * 64 + (el & 63)] |= 1ull << (el >> 6);
            }
        e = hipMemcpy(c->sgn, words.data(), words.size() * sizeof(uint32_t), hipMemcpyHostToDevice);
        if (e == hipSuccess)
            e = hipMemcpy(c->sgn_lane, lanes.data(), lanes.size() * sizeof(u64), hipMemcpyHostToDevice);
    }
    if (e == hipSuccess) e = hipMemcpy(c->Wt, Wt.data(), Wt.size() * sizeof(float), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(c->wb, wb.data(), wb.size() * sizeof(float), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemset(c->counts, 0, (size_t)(c->cbits / 8) * (size_t)L * B);
    if (e == hipSuccess) e = hipMemset(c->S2, 0, sizeof(u64) * (size_t)L);
    if (e == hipSuccess) e = hipMemset(c->S3, 0, sizeof(u64) * 2 * (size_t)L);
    if (e == hipSuccess) e = hipMemset(c->mom, 0, sizeof(u64) * 4);
    if (e == hipSuccess) e = hipMemset(c->rcnt, 0, sizeof(u64) * 4);
    if (e == hipSuccess) e = hipMemset(c->err, 0, sizeof(unsigned) * 4);
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e != hipSuccess) {
        (void)hipGetLastError();
        free_all(c);
        delete c;
        return ACE_E_DEVICE;
    }
    *out = c;
    return ACE_OK;
}

}  // namespace

ace_status ace_destroy(ace_ctx c) {
    if (!c) return ACE_OK;
    if (c->server_attached) return ACE_E_STATE;
    DeviceGuard g(c->cfg.device);
    (void)hipDeviceSynchronize();
    free_all(c);
    delete c;
    return ACE_OK;
}

ace_status ace_reset(ace_ctx c, void* stream) {
    ace_status st = enter(c);
    if (st) return st;
    if (take_injected_failure(c)) return ACE_E_DEVICE;
    DeviceGuard g(c->cfg.device);
    hipStream_t s = (hipStream_t)stream;
    Bracket br(c, s, CLS_OTHER);
    const size_t cb = (size_t)(c->cbits / 8) * (size_t)c->cfg.L << c->cfg.K;
    st = check(c, launch_zero_with_small(c->counts, cb, c->rcnt + 3, 1, c->S2, c->cfg.L, c->S3, 2 * (int64_t)c->cfg.L,
                                         c->mom, 4, s));
    if (!st) c->n_total = 0;
    return st;
}

ace_status ace_reset_scored(ace_ctx c, void* stream) {
    ace_status st = enter(c);
    if (st) return st;
    if (take_injected_failure(c)) return ACE_E_DEVICE;
    DeviceGuard g(c->cfg.device);
    return check(c, launch_zero(c->mom, sizeof(u64) * 4, (hipStream_t)stream));
}

ace_status ace_insert(ace_ctx c, const float* X, int64_t n, void* stream) {
    ace_status st = enter(c);
    if (st) return st;
    if (n < 0 || (n > 0 && !X)) return ACE_E_INVALID;
    if (n == 0) return ACE_OK;
    if (c->n_total + n > c->cap) return ACE_E_OVERFLOW;
    if (take_injected_failure(c)) return ACE_E_DEVICE;
    DeviceGuard g(c->cfg.device);
    st = update_rows(c, X, n, +1, (hipStream_t)stream);
    if (!st) c->n_total += n;
    return st;
}

ace_status ace_delete(ace_ctx c, const float* X, int64_t n, void* stream) {
    ace_status st = enter(c);
    if (st) return st;
    if (n < 0 || (n > 0 && !X)) return ACE_E_INVALID;
    if (n == 0) return ACE_OK;
    if (n > c->n_total) return ACE_E_STATE;
    if (take_injected_failure(c)) return ACE_E_DEVICE;
    DeviceGuard g(c->cfg.device);
    st = update_rows(c, X, n, -1, (hipStream_t)stream);
    if (!st) c->n_total -= n;
    return st;
}

ace_status ace_insert_codes(ace_ctx c, const uint16_t* codes, int64_t n, void* stream) {
    ace_status st = enter(c);
    if (st) return st;
    if (n < 0 || (n > 0 && !codes)) return ACE_E_INVALID;
    if (n == 0) return ACE_OK;
    if (c->n_total + n > c->cap) return ACE_E_OVERFLOW;
    if (take_injected_failure(c)) return ACE_E_DEVICE;
    DeviceGuard g(c->cfg.device);
    st = check(c, launch_count_update(codes, n, n, c->cfg.K, c->cfg.L, +1, c->counts, c->cbits, c->S2, c->S3, c->err,
                                      c->rcnt + 3,
                                      (hipStream_t)stream));
    if (!st) c->n_total += n;
    return st;
}

static ace_status score_guard(ace_ctx c) {
    // T = sum of L counts, each <= n_total (and <= 65535 with 16-bit counters), must fit uint32.
    if (c->cbits == 32 && (u64)c->cfg.L * (u64)c->n_total > 0xFFFFFFFFull) return ACE_E_OVERFLOW;
    return ACE_OK;
}

ace_status ace_score(ace_ctx c, const float* X, int64_t n, float* s_out, uint32_t* T_out, void* stream) {
    ace_status st = enter(c);
    if (st) return st;
    if (n < 0 || (n > 0 && !X)) return ACE_E_INVALID;
    if (n == 0) return ACE_OK;
    if ((st = score_guard(c))) return st;
    if (take_injected_failure(c)) return ACE_E_DEVICE;
    DeviceGuard g(c->cfg.device);
    hipStream_t s = (hipStream_t)stream;
    for (int64_t r0 = 0; r0 < n; r0 += c->ws_rows) {
        const int64_t m = (n - r0 < c->ws_rows) ? n - r0 : c->ws_rows;
        st = hash_chunk(c, &c->ws, X + r0 * (int64_t)c->cfg.d, m, false, s);
        if (st) return st;
        {
            Bracket br(c, s, CLS_SCORE, m);
            st = check(c, launch_score(c->ws.codes, m, m, c->cfg.K, c->cfg.L, c->counts, c->cbits,
                                       s_out ? s_out + r0 : nullptr, T_out ? T_out + r0 : nullptr, c->mom, s,
                                       c->mpart, c->mpart_cap));
        }
        if (st) return st;
    }
    return ACE_OK;
}

ace_status ace_score_codes(ace_ctx c, const uint16_t* codes, int64_t n, float* s_out, uint32_t* T_out,
                           void* stream) {
    ace_status st = enter(c);
    if (st) return st;
    if (n < 0 || (n > 0 && !codes)) return ACE_E_INVALID;
    if (n == 0) return ACE_OK;
    if ((st = score_guard(c))) return st;
    if (take_injected_failure(c)) return ACE_E_DEVICE;
    DeviceGuard g(c->cfg.device);
    return check(c, launch_score(codes, n, n, c->cfg.K, c->cfg.L, c->counts, c->cbits, s_out, T_out, c->mom,
                                 (hipStream_t)stream, c->mpart, c->mpart_cap));
}

ace_status ace_hash(ace_ctx c, const float* X, int64_t n, uint16_t* codes, uint16_t* refined, void* stream) {
    ace_status st = enter(c);
    if (st) return st;
    if (n < 0 || (n > 0 && (!X || !codes))) return ACE_E_INVALID;
    if (n == 0) return ACE_OK;
    DeviceGuard g(c->cfg.device);
    if (refined && !c->ws.refined) {
        st = dev_alloc(c, (void**)&c->ws.refined, sizeof(uint16_t) * ((size_t)c->cfg.L * c->ws_rows + 2));
        if (st) return st;
    }
    if (take_injected_failure(c)) return ACE_E_DEVICE;
    hipStream_t s = (hipStream_t)stream;
    const size_t L = (size_t)c->cfg.L;
    for (int64_t r0 = 0; r0 < n; r0 += c->ws_rows) {
        const int64_t m = (n - r0 < c->ws_rows) ? n - r0 : c->ws_rows;
        st = hash_chunk(c, &c->ws, X + r0 * (int64_t)c->cfg.d, m, refined != nullptr, s);
        if (st) return st;
        // Workspace [L][m] -> caller's [L][n] at column r0.
        st = check(c, hipMemcpy2DAsync(codes + r0, sizeof(uint16_t) * n, c->ws.codes, sizeof(uint16_t) * m,
                                       sizeof(uint16_t) * m, L, hipMemcpyDeviceToDevice, s));
        if (!st && refined)
            st = check(c, hipMemcpy2DAsync(refined + r0, sizeof(uint16_t) * n, c->ws.refined, sizeof(uint16_t) * m,
                                           sizeof(uint16_t) * m, L, hipMemcpyDeviceToDevice, s));
        if (st) return st;
    }
    return ACE_OK;
}

ace_status ace_threshold(ace_ctx c, int32_t mode, double alpha, void* stream, ace_thresh* out) {
    ace_status st = enter(c);
    if (st) return st;
    if (!out || mode < 0 || mode > 2 || !isfinite(alpha)) return ACE_E_INVALID;
    if (take_injected_failure(c)) return ACE_E_DEVICE;
    DeviceGuard g(c->cfg.device);
    hipStream_t s = (hipStream_t)stream;
    {
        Bracket br(c, s, CLS_OTHER);
        st = check(c, launch_threshold(c->n_total, c->cfg.L, c->S2, c->S3, c->mom, c->err, mode, alpha, c->thr_dev,
                                       s));
    }
    if (st) return st;
    if ((st = check(c, hipStreamSynchronize(s)))) return st;
    const DevThresh r = *c->thr;
    if (r.err) {
        c->sticky = ACE_E_STATE;
        return ACE_E_STATE;
    }
    out->n = r.n;
    out->m_scored = r.m_scored;
    out->mu = r.mu;
    out->mu_scored = r.mu_scored;
    out->sigma = r.sigma;
    out->sigma_table = r.sigma_table;
    out->tau = r.tau;
    out->mode = r.mode;
    out->pad = 0;
    return r.status ? (ace_status)r.status : ACE_OK;
}

ace_status ace_threshold_flag(ace_ctx c, int32_t mode, double alpha, const uint32_t* T, int64_t n, uint8_t* flags,
                              void* stream, ace_thresh* out) {
    ace_status st = enter(c);
    if (st) return st;
    if (!out || mode < 0 || mode > 2 || !isfinite(alpha) || n < 0 || (n > 0 && (!T || !flags))) return ACE_E_INVALID;
    if (take_injected_failure(c)) return ACE_E_DEVICE;
    DeviceGuard g(c->cfg.device);
    hipStream_t s = (hipStream_t)stream;
    {
        Bracket br(c, s, CLS_OTHER);
        st = check(c, launch_threshold(c->n_total, c->cfg.L, c->S2, c->S3, c->mom, c->err, mode, alpha, c->thr_dev,
                                       s, c->lim));
        if (!st) st = check(c, launch_flags_dev(T, n, c->lim, mode, flags, s));
    }
    if (st) return st;
    if ((st = check(c, hipStreamSynchronize(s)))) return st;
    const DevThresh r = *c->thr;
    if (r.err) {
        c->sticky = ACE_E_STATE;
        return ACE_E_STATE;
    }
    out->n = r.n;
    out->m_scored = r.m_scored;
    out->mu = r.mu;
    out->mu_scored = r.mu_scored;
    out->sigma = r.sigma;
    out->sigma_table = r.sigma_table;
    out->tau = r.tau;
    out->mode = r.mode;
    out->pad = 0;
    return r.status ? (ace_status)r.status : ACE_OK;
}

ace_status ace_flag(ace_ctx c, const uint32_t* T, int64_t n, double tau, int32_t mode, uint8_t* flags, void* stream) {
    ace_status st = enter(c);
    if (st) return st;
    if (n < 0 || mode < 0 || mode > 2 || !isfinite(tau) || (n > 0 && (!T || !flags))) return ACE_E_INVALID;
    if (n == 0) return ACE_OK;
    if (take_injected_failure(c)) return ACE_E_DEVICE;
    DeviceGuard g(c->cfg.device);
    Bracket br(c, (hipStream_t)stream, CLS_OTHER);
    return check(c, launch_flags(T, n, c->cfg.L, tau, mode, flags, (hipStream_t)stream));
}

static ace_status sync_and_check(ace_ctx c) {
    hipError_t e = hipDeviceSynchronize();
    ace_status st = check(c, e);
    if (st) return st;
    unsigned errs[4];
    if ((st = check(c, hipMemcpy(errs, c->err, sizeof(errs), hipMemcpyDeviceToHost)))) return st;
    if (errs[0]) {
        c->sticky = ACE_E_STATE;
        return ACE_E_STATE;
    }
    return ACE_OK;
}

ace_status ace_get_counts(ace_ctx c, int32_t* host) {
    ace_status st = enter(c);
    if (st) return st;
    if (!host) return ACE_E_INVALID;
    DeviceGuard g(c->cfg.device);
    if ((st = sync_and_check(c))) return st;
    const size_t cnt = (size_t)c->cfg.L << c->cfg.K;
    if (c->cbits == 32) return check(c, hipMemcpy(host, c->counts, sizeof(int32_t) * cnt, hipMemcpyDeviceToHost));
    std::vector<uint16_t> tmp(cnt);
    st = check(c, hipMemcpy(tmp.data(), c->counts, sizeof(uint16_t) * cnt, hipMemcpyDeviceToHost));
    if (!st)
        for (size_t i = 0; i < cnt; ++i) host[i] = tmp[i];
    return st;
}

ace_status ace_get_table_stats(ace_ctx c, int64_t* S2_host, uint64_t* S3_host) {
    ace_status st = enter(c);
    if (st) return st;
    if (!S2_host || !S3_host) return ACE_E_INVALID;
    DeviceGuard g(c->cfg.device);
    if ((st = sync_and_check(c))) return st;
    st = check(c, hipMemcpy(S2_host, c->S2, sizeof(u64) * (size_t)c->cfg.L, hipMemcpyDeviceToHost));
    if (st) return st;
    return check(c, hipMemcpy(S3_host, c->S3, sizeof(u64) * 2 * (size_t)c->cfg.L, hipMemcpyDeviceToHost));
}

ace_status ace_get_memory(ace_ctx c, int64_t* bytes) {
    if (!c || !bytes) return ACE_E_INVALID;
    *bytes = (int64_t)c->bytes;
    return ACE_OK;
}

ace_status ace_get_counters(ace_ctx c, ace_counters* out) {
    ace_status st = enter(c);
    if (st) return st;
    if (!out) return ACE_E_INVALID;
    DeviceGuard g(c->cfg.device);
    if ((st = sync_and_check(c))) return st;
    u64 mom[4], r[4];
    st = check(c, hipMemcpy(mom, c->mom, sizeof(mom), hipMemcpyDeviceToHost));
    if (!st) st = check(c, hipMemcpy(r, c->rcnt, sizeof(r), hipMemcpyDeviceToHost));
    if (st) return st;
    out->n = c->n_total;
    out->m_scored = (int64_t)mom[0];
    out->sum_T = (int64_t)mom[1];
    out->sum_T2_lo = mom[2];
    out->sum_T2_hi = mom[3];
    out->bits_hashed = c->bits_hashed;
    out->bits_refined = r[0];
    out->bits_flipped = r[1];
    out->bits_in_bound_unrefined = r[2];
    out->saturated_increments = r[3];
    return ACE_OK;
}

ace_status ace_exact_score(const float* Q, int64_t m, const float* X, int64_t n, int32_t d, int32_t K, double* S,
                           double* S2, int32_t device, void* stream) {
    if (m < 0 || n < 0 || d < 1 || K < 1 || K > 64 || device < 0) return ACE_E_INVALID;
    if (m > 0 && (!Q || !S)) return ACE_E_INVALID;
    if (n > 0 && !X) return ACE_E_INVALID;
    if ((int64_t)d > (int64_t)1 << 24) return ACE_E_INVALID;
    if (m == 0) return ACE_OK;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device >= ndev) {
        (void)hipGetLastError();
        return ACE_E_DEVICE;
    }
    DeviceGuard g(device);
    if (!g.ok) return ACE_E_DEVICE;
    hipError_t e = launch_exact_score(Q, m, X, n, d, K, S, S2, (hipStream_t)stream);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return ACE_E_DEVICE;
    }
    return ACE_OK;
}

ace_status ace_set_counts(ace_ctx c, const int32_t* host, int64_t n) {
    ace_status st = enter(c);
    if (st) return st;
    if (!host || n < 0 || n > c->cap) return ACE_E_INVALID;
    const int64_t B = (int64_t)1 << c->cfg.K;
    const int32_t top = c->cbits == 16 ? 65535 : INT32_MAX;
    for (int j = 0; j < c->cfg.L; ++j) {
        int64_t sum = 0;
        for (int64_t b = 0; b < B; ++b) {
            if (host[(int64_t)j * B + b] < 0 || host[(int64_t)j * B + b] > top) return ACE_E_INVALID;
            sum += host[(int64_t)j * B + b];
        }
        // saturated 16-bit counts may sum to less than n (dropped increments)
        if (c->cbits == 32 ? sum != n : sum > n) return ACE_E_INVALID;
    }
    DeviceGuard g(c->cfg.device);
    if ((st = sync_and_check(c))) return st;
    if (c->cbits == 32) {
        st = check(c, hipMemcpy(c->counts, host, sizeof(int32_t) * (size_t)c->cfg.L * B, hipMemcpyHostToDevice));
    } else {
        std::vector<uint16_t> tmp((size_t)c->cfg.L * B);
        for (size_t i = 0; i < tmp.size(); ++i) tmp[i] = (uint16_t)host[i];
        st = check(c, hipMemcpy(c->counts, tmp.data(), sizeof(uint16_t) * tmp.size(), hipMemcpyHostToDevice));
    }
    if (!st) st = check(c, launch_table_sums(c->counts, c->cbits, c->cfg.K, c->cfg.L, c->S2, c->S3, nullptr));
    if (!st) st = check(c, launch_zero(c->mom, sizeof(u64) * 4, nullptr));
    if (!st) st = check(c, hipDeviceSynchronize());
    if (!st) c->n_total = n;
    return st;
}

ace_status ace_profile_enable(ace_ctx c, int32_t on) {
    if (!c) return ACE_E_INVALID;
    c->profiling = on ? 1 : 0;
    return ACE_OK;
}

ace_status ace_get_profile(ace_ctx c, ace_profile* out) {
    ace_status st = enter(c);
    if (st) return st;
    if (!out) return ACE_E_INVALID;
    DeviceGuard g(c->cfg.device);
    if ((st = check(c, hipDeviceSynchronize()))) return st;
    memset(out, 0, sizeof(*out));
    for (auto& t : c->timed) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, t.a, t.b) != hipSuccess) {
            (void)hipGetLastError();
            ms = 0.f;
        }
        switch (t.cls) {
            case CLS_HASH: out->hash_ms += ms; out->hash_launches++; out->hash_rows += t.rows; break;
            case CLS_UPDATE: out->update_ms += ms; out->update_launches++; break;
            case CLS_SCORE: out->score_ms += ms; out->score_launches++; break;
            case CLS_REFINE: out->refine_ms += ms; out->refine_launches++; break;
            case CLS_CONVERT: out->convert_ms += ms; out->convert_launches++; break;
            default: out->other_ms += ms; out->other_launches++; break;
        }
        c->pool.push_back(t.a);
        c->pool.push_back(t.b);
    }
    c->timed.clear();
    return ACE_OK;
}

ace_status ace_debug_fail_next(ace_ctx c) {
    if (!c) return ACE_E_INVALID;
    c->fail_next = 1;
    return ACE_OK;
}

ace_status ace_debug_set_refine_queue(ace_ctx c, int64_t entries) {
    if (!c || entries < 0) return ACE_E_INVALID;
    c->list_cap = (entries == 0 || (u64)entries > c->ws.list_alloc) ? c->ws.list_alloc : (u64)entries;
    return ACE_OK;
}

ace_status ace_debug_set_capacity(ace_ctx c, int64_t max_points) {
    if (!c || max_points < 0) return ACE_E_INVALID;
    c->cap = max_points == 0 ? (int64_t)INT32_MAX : max_points;
    return ACE_OK;
}

}  // extern "C"
