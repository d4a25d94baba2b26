// Allocation-free hashing: ace_hash_static, the variant of ace_hash whose scratch (queue of
// uncertain projections, its counter, the code and refined-mask staging, the converted
// low-precision rows and their norms) lives in one file-scope device array per GPU instead
// of the context's workspace.  For callers that cannot allocate device memory (HIP graph
// capture, tight serving loops): it calls no hipMalloc or hipFree and nothing that does.
#include <mutex>

#include "ace_context.h"

using namespace ace;

namespace {
constexpr size_t kScratchBytes = (size_t)64 << 20;   // per GPU, held until the process ends
}  // namespace

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

constexpr int kMaxDevices = 64;
constexpr int64_t kChunkStep = 256;                   // chunk rows are a multiple of this

// Device address of each GPU's copy of `scratch` (host code must never pass the symbol
// itself to a kernel or a copy: on the host it is only a stand-in).
std::mutex g_mu;
void* g_scratch[kMaxDevices] = {};

size_t align256(size_t b) { return (b + 255) / 256 * 256; }

struct Layout {
    size_t codes = 0, refined = 0, list = 0, list_count = 0, xh = 0, xl = 0, xq = 0, rown = 0, end = 0;
    u64 list_alloc = 0;
};

// Byte offsets inside the scratch array for chunks of m rows (same sizes as the context's
// workspace for m rows: ws_alloc).
Layout layout_for(ace_ctx c, int64_t m) {
    Layout o;
    const size_t L = (size_t)c->cfg.L;
    const size_t rows16 = (size_t)(m + 15) / 16 * 16;
    size_t p = 0;
    o.codes = p;
    p += align256(sizeof(uint16_t) * (L * (size_t)m + 2));
    o.refined = p;
    p += align256(sizeof(uint16_t) * (L * (size_t)m + 2));
    o.list_alloc = (u64)m * (u64)L * KPAD / 32;
    if (o.list_alloc < 65536) o.list_alloc = 65536;
    o.list = p;
    p += align256(sizeof(u64) * (size_t)o.list_alloc);
    o.list_count = p;
    p += align256(sizeof(u64));
    if (c->cfg.precision == ACE_BF16) {
        o.xh = p;
        p += align256(sizeof(uint16_t) * rows16 * (size_t)c->DP);
        o.xl = p;
        p += align256(sizeof(uint16_t) * rows16 * (size_t)c->DP);
    }
    if (c->cfg.precision == ACE_FP8E4M3) {
        o.xq = p;
        p += align256(rows16 * (size_t)c->DP);
    }
    if (c->cfg.precision != ACE_FP32) {
        o.rown = p;
        p += align256(sizeof(float) * 3 * (size_t)m);
    }
    o.end = p;
    return o;
}

// Largest chunk (a multiple of kChunkStep rows) whose layout fits the array; 0 if not even
// kChunkStep rows fit.
int64_t chunk_rows(ace_ctx c) {
    // the codes and refined-mask staging alone take 4 L bytes per row
    int64_t lo = 0, hi = (int64_t)(kScratchBytes / (4 * (size_t)c->cfg.L)) / kChunkStep;
    while (lo < hi) {   // largest k in [0, hi] with layout_for(k * step) fitting
        const int64_t mid = (lo + hi + 1) / 2;
        if (layout_for(c, mid * kChunkStep).end <= kScratchBytes) lo = mid;
        else hi = mid - 1;
    }
    return lo * kChunkStep;
}

struct DevSwitch {
    int prev = -1;
    bool ok = true;
    explicit DevSwitch(int dev) {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        ok = hipSetDevice(dev) == hipSuccess;
    }
    ~DevSwitch() {
        if (prev >= 0) (void)hipSetDevice(prev);
    }
};

}  // namespace

// Resolve the address of `scratch` on `device` (which must be current), once per device.
// Called by context creation, and by ace_hash_static if creation did not manage it.
ace_status ace::scratch_bind(int device) {
    if (device < 0 || device >= kMaxDevices) return ACE_E_INVALID;
    std::lock_guard<std::mutex> lk(g_mu);
    if (g_scratch[device]) return ACE_OK;
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
        (void)hipGetLastError();
        return ACE_E_DEVICE;
    }
    g_scratch[device] = p;
    return ACE_OK;
}

extern "C" ace_status ace_hash_static(ace_ctx c, const float* X, int64_t n, uint16_t* codes, uint16_t* refined,
                                      void* stream) {
    if (!c) return ACE_E_INVALID;
    if (c->sticky != ACE_OK) return c->sticky;
    if (n < 0 || (n > 0 && (!X || !codes))) return ACE_E_INVALID;
    const int64_t m_max = chunk_rows(c);
    if (m_max < kChunkStep) return ACE_E_INVALID;   // one chunk of this context's rows does not fit
    if (n == 0) return ACE_OK;
    DevSwitch g(c->cfg.device);
    if (!g.ok) return ACE_E_DEVICE;
    void* base = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        base = g_scratch[c->cfg.device];
    }
    if (!base) {
        const ace_status st = scratch_bind(c->cfg.device);
        if (st) return st;
        std::lock_guard<std::mutex> lk(g_mu);
        base = g_scratch[c->cfg.device];
    }
    unsigned char* b = static_cast<unsigned char*>(base);
    const Layout o = layout_for(c, m_max);
    Workspace w;
    w.rows = m_max;
    w.codes = reinterpret_cast<uint16_t*>(b + o.codes);
    w.refined = reinterpret_cast<uint16_t*>(b + o.refined);
    w.list = reinterpret_cast<u64*>(b + o.list);
    w.list_count = reinterpret_cast<u64*>(b + o.list_count);
    w.list_alloc = o.list_alloc;
    if (o.xh) {
        w.xh = reinterpret_cast<uint16_t*>(b + o.xh);
        w.xl = reinterpret_cast<uint16_t*>(b + o.xl);
    }
    if (o.xq) w.xq = b + o.xq;
    if (o.rown) w.rown = reinterpret_cast<float*>(b + o.rown);
    hipStream_t s = (hipStream_t)stream;
    const size_t L = (size_t)c->cfg.L;
    for (int64_t r0 = 0; r0 < n; r0 += m_max) {
        const int64_t m = (n - r0 < m_max) ? n - r0 : m_max;
        // hash_chunk zeroes the queue counter (and the refined mask) with fill kernels first
        ace_status st = hash_chunk(c, &w, X + r0 * (int64_t)c->cfg.d, m, refined != nullptr, s);
        if (st) return st;
        st = check(c, hipMemcpy2DAsync(codes + r0, sizeof(uint16_t) * n, w.codes, sizeof(uint16_t) * m,
                                       sizeof(uint16_t) * m, L, hipMemcpyDeviceToDevice, s));
        if (!st && refined)
            st = check(c, hipMemcpy2DAsync(refined + r0, sizeof(uint16_t) * n, w.refined, sizeof(uint16_t) * m,
                                           sizeof(uint16_t) * m, L, hipMemcpyDeviceToDevice, s));
        if (st) return st;
    }
    return ACE_OK;
}
