// Exact target of the ACE estimator (Sec. 3, Eq. thescore):
//   S(q, D) = sum_{x in D} p(q, x)^K,   p = 1 - theta / pi,  theta = arccos(q.x / (|q| |x|)),
// the SRP collision probability of one bit (Sec. 2.1, Eq. srp) raised to the K bits of a
// code.  Theorem 1 states that every table's count at the query's bucket has mean S(q, D).
// Zero vectors: p = 1 when both are zero, 1/2 when one is (every bit of a zero vector is 0,
// every bit of a nonzero one is a fair coin).
//
// One launch: a grid of 64-query x (64 * XT)-point blocks.  The inner products q.x and the
// squared norms are FP64 sums of exact FP64 products of the FP32 inputs, accumulated on
// v_mfma_f64_16x16x4f64 (products of FP32 values are exact in FP64, so the only error is
// the FP64 summation).  The epilogue turns each inner product into p^K in FP64 and sums
// the block's points per query (the wave's inner products pass through LDS so that each
// lane walks 16 points of one query in a rolled loop); one FP64 atomic per query and
// wave adds the partial sum into S (order of those additions unspecified).  Optionally the same for
// sum p^{2K}, which gives the variance of uniform sampling (Sec. 3, Theorem 2's RSE).
//
// 256 threads = 4 waves as 2 (queries) x 2 (points); a wave owns 32 x 32 outputs as
// 2 x 2 MFMA tiles.  Operands go through LDS in chunks of 64 rows x 64 columns (coalesced
// reads, row stride 68 floats so the fragment reads of a wave hit distinct banks).  The
// cosine is the inner product times the two inverse norms (1 / sqrt of the FP64 squared
// norms, each computed once per row and tile).
#include "ace_internal.h"

namespace ace {

namespace {

typedef double d4 __attribute__((ext_vector_type(4)));

constexpr int XT = 8;     // point tiles per workgroup
constexpr int BK = 64;    // contraction chunk staged in LDS
constexpr int LDR = BK + 4;   // LDS row stride (floats): fragment reads hit 64 distinct banks

__device__ inline double pow_int(double p, int K) {
    double r = 1.0, b = p;
    for (int e = K; e > 0; e >>= 1) {
        if (e & 1) r *= b;
        b *= b;
    }
    return r;
}

// Stage rows [r0, r0 + 64) x columns [k0, k0 + BK) of A (FP32 [rows][d]) into T, zero
// outside the matrix.  Consecutive threads read consecutive columns of a row; VEC (d a
// multiple of 4, A 16-byte aligned) reads 16 bytes per thread.
template <bool VEC>
__device__ inline void stage(float* __restrict__ T, const float* __restrict__ A, int64_t rows, int d, int64_t r0,
                             int k0) {
    if (VEC) {
        typedef float f4 __attribute__((ext_vector_type(4)));
#pragma unroll 2
        for (int s = 0; s < (64 * BK) / (4 * 256); ++s) {
            const int idx = threadIdx.x + 256 * s;
            const int r = idx / (BK / 4), k = 4 * (idx % (BK / 4));
            const int64_t gr = r0 + r;
            const int gk = k0 + k;
            f4 v = f4{0.f, 0.f, 0.f, 0.f};
            if (gr < rows && gk < d) v = *reinterpret_cast<const f4*>(A + gr * (int64_t)d + gk);   // d % 4 == 0
            *reinterpret_cast<f4*>(T + r * LDR + k) = v;
        }
    } else {
#pragma unroll 2
        for (int s = 0; s < (64 * BK) / 256; ++s) {
            const int idx = threadIdx.x + 256 * s;
            const int r = idx / BK, k = idx % BK;
            const int64_t gr = r0 + r;
            const int gk = k0 + k;
            T[r * LDR + k] = (gr < rows && gk < d) ? A[gr * (int64_t)d + gk] : 0.f;
        }
    }
}

// Per-wave epilogue area, aliased onto the staging buffer once a tile's contraction is
// done: the 32 x 32 inner products (row stride 33 doubles against bank conflicts) and
// the inverse norms of the wave's 32 queries and 32 points (0 marks a zero vector).
constexpr int ER = 33;
constexpr int EW = 32 * ER + 64;                       // doubles per wave
constexpr int STAGE_BYTES = 2 * 64 * LDR * 4;
constexpr int EPI_BYTES = 4 * EW * 8;
constexpr int BUF_BYTES = STAGE_BYTES > EPI_BYTES ? STAGE_BYTES : EPI_BYTES;

template <bool WANT_S2, bool VEC>
__global__ __launch_bounds__(256) void exact_score_kernel(const float* __restrict__ Q, int64_t m,
                                                          const float* __restrict__ X, int64_t n, int d, int K,
                                                          double* __restrict__ S, double* __restrict__ S2) {
    __shared__ double buf[BUF_BYTES / 8];
    float* Qs = reinterpret_cast<float*>(buf);
    float* Xs = Qs + 64 * LDR;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int wm = wave >> 1, wn = wave & 1;
    const int64_t qb = (int64_t)blockIdx.y * 64;
    const int64_t xblk = (int64_t)blockIdx.x * 64 * XT;
    const int lr = lane & 15, lk = lane >> 4;
    double* E = buf + wave * EW;           // this wave's epilogue area
    double* inv_q = E + 32 * ER;
    double* inv_x = inv_q + 32;
    // Epilogue ownership: lane -> query row erow of the wave, points ec0 .. ec0 + 15.
    const int erow = lane >> 1, ec0 = (lane & 1) * 16;
    const bool qin = qb + wm * 32 + erow < m;
    double part = 0.0, part2 = 0.0;

    for (int t = 0; t < XT; ++t) {
        const int64_t xb = xblk + (int64_t)t * 64;
        if (xb >= n) break;   // uniform over the workgroup
        d4 acc[2][2];
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j) acc[i][j] = d4{0.0, 0.0, 0.0, 0.0};
        double qq[2] = {0.0, 0.0}, xx[2] = {0.0, 0.0};
        for (int k0 = 0; k0 < d; k0 += BK) {
            __syncthreads();
            stage<VEC>(Qs, Q, m, d, qb, k0);
            stage<VEC>(Xs, X, n, d, xb, k0);
            __syncthreads();
#pragma unroll 4
            for (int kk = 0; kk < BK; kk += 4) {
                double a[2], b[2];
#pragma unroll
                for (int i = 0; i < 2; ++i) {
                    a[i] = (double)Qs[(wm * 32 + 16 * i + lr) * LDR + kk + lk];
                    qq[i] += a[i] * a[i];
                }
#pragma unroll
                for (int j = 0; j < 2; ++j) {
                    b[j] = (double)Xs[(wn * 32 + 16 * j + lr) * LDR + kk + lk];
                    xx[j] += b[j] * b[j];
                }
#pragma unroll
                for (int i = 0; i < 2; ++i)
#pragma unroll
                    for (int j = 0; j < 2; ++j)
                        acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], b[j], acc[i][j], 0, 0, 0);
            }
        }
        // Squared norms: lanes lr, lr+16, lr+32, lr+48 hold the four k phases of row lr.
#pragma unroll
        for (int i = 0; i < 2; ++i) {
            qq[i] += __shfl_xor(qq[i], 16, 64);
            qq[i] += __shfl_xor(qq[i], 32, 64);
            xx[i] += __shfl_xor(xx[i], 16, 64);
            xx[i] += __shfl_xor(xx[i], 32, 64);
        }
        __syncthreads();   // every wave is done reading the staged operands
        // Tile (i, j), reg r of lane l: query 16i + lk + 4r, point 16j + lr of the wave.
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j)
#pragma unroll
                for (int r = 0; r < 4; ++r) E[(16 * i + lk + 4 * r) * ER + 16 * j + lr] = acc[i][j][r];
        if (lk == 0) {
#pragma unroll
            for (int i = 0; i < 2; ++i) {
                inv_q[16 * i + lr] = qq[i] > 0.0 ? 1.0 / sqrt(qq[i]) : 0.0;
                inv_x[16 * i + lr] = xx[i] > 0.0 ? 1.0 / sqrt(xx[i]) : 0.0;
            }
        }
        __syncthreads();
        const double iq = inv_q[erow];
        const int64_t x0 = xb + wn * 32;
        for (int c = ec0; c < ec0 + 16; ++c) {
            const double ix = inv_x[c];
            double p;
            if (iq == 0.0 && ix == 0.0) {
                p = 1.0;
            } else if (iq == 0.0 || ix == 0.0) {
                p = 0.5;
            } else {
                double cs = E[erow * ER + c] * iq * ix;
                cs = cs > 1.0 ? 1.0 : (cs < -1.0 ? -1.0 : cs);
                p = 1.0 - acos(cs) * 0.3183098861837907;   // 1 / pi
            }
            const double v = (qin && x0 + c < n) ? pow_int(p, K) : 0.0;
            part += v;
            if (WANT_S2) part2 += v * v;
        }
    }
    part += __shfl_xor(part, 1, 64);
    if (WANT_S2) part2 += __shfl_xor(part2, 1, 64);
    if ((lane & 1) == 0 && qin) {
        const int64_t q = qb + wm * 32 + erow;
        atomicAdd(&S[q], part);
        if (WANT_S2) atomicAdd(&S2[q], part2);
    }
}

}  // namespace

hipError_t launch_exact_score(const float* Q, int64_t m, const float* X, int64_t n, int d, int K, double* S,
                              double* S2, hipStream_t s) {
    hipError_t e = launch_zero(S, sizeof(double) * (size_t)m, s);
    if (e == hipSuccess && S2) e = launch_zero(S2, sizeof(double) * (size_t)m, s);
    if (e != hipSuccess || n == 0) return e;
    const int64_t gx = (n + 64 * XT - 1) / (64 * XT), gy = (m + 63) / 64;
    const bool vec = d % 4 == 0 && (reinterpret_cast<uintptr_t>(Q) & 15u) == 0 &&
                     (reinterpret_cast<uintptr_t>(X) & 15u) == 0;
    const dim3 grid((unsigned)gx, (unsigned)gy);
    if (S2 && vec)
        hipLaunchKernelGGL((exact_score_kernel<true, true>), grid, dim3(256), 0, s, Q, m, X, n, d, K, S, S2);
    else if (S2)
        hipLaunchKernelGGL((exact_score_kernel<true, false>), grid, dim3(256), 0, s, Q, m, X, n, d, K, S, S2);
    else if (vec)
        hipLaunchKernelGGL((exact_score_kernel<false, true>), grid, dim3(256), 0, s, Q, m, X, n, d, K, S, S2);
    else
        hipLaunchKernelGGL((exact_score_kernel<false, false>), grid, dim3(256), 0, s, Q, m, X, n, d, K, S, S2);
    return hipGetLastError();
}

}  // namespace ace
