// Diagnostic of the matrix-unit arithmetic that the measured refinement bound assumes
// (the sign of every projection must be that of the exact sum outside the bound, Sec. 2.1).
// One wave runs ONE instruction D = C + A B on hand-built operands, so a caller can check
// the rounding, order and alignment the bound charges for, on the device at hand.
//
// Operand positions: lane l supplies row (or column) l mod 16 and the KL consecutive k
// values KL (l / 16) .. KL (l / 16) + KL - 1 (KL = 1 FP32, 8 BF16, 32 e4m3), the same k for
// both operands, as the projection kernels' operand tiles do.  D and C: lane l, element i
// is row 4 (l / 16) + i, column l mod 16.
#include "ace_internal.h"

namespace ace {

namespace {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef short s8v __attribute__((ext_vector_type(8)));
typedef int i8v __attribute__((ext_vector_type(8)));

template <int KIND>
__global__ __launch_bounds__(64) void mfma_probe_kernel(const void* __restrict__ A, const void* __restrict__ B,
                                                        const float* __restrict__ C, float* __restrict__ D) {
    const int l = threadIdx.x, r = l & 15, g = l >> 4;
    f4 c;
#pragma unroll
    for (int i = 0; i < 4; ++i) c[i] = C[(4 * g + i) * 16 + r];
    f4 d;
    if constexpr (KIND == 0) {
        const float a = reinterpret_cast<const float*>(A)[r * 4 + g];
        const float b = reinterpret_cast<const float*>(B)[g * 16 + r];
        d = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    } else if constexpr (KIND == 1) {
        const uint16_t* a16 = reinterpret_cast<const uint16_t*>(A);
        const uint16_t* b16 = reinterpret_cast<const uint16_t*>(B);
        s8v av, bv;
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            av[i] = (short)a16[r * 32 + 8 * g + i];
            bv[i] = (short)b16[(8 * g + i) * 16 + r];
        }
        d = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf8, av), __builtin_bit_cast(bf8, bv), c, 0,
                                                     0, 0);
    } else {
        const uint8_t* a8 = reinterpret_cast<const uint8_t*>(A);
        const uint8_t* b8 = reinterpret_cast<const uint8_t*>(B);
        i8v av, bv;
#pragma unroll
        for (int w = 0; w < 8; ++w) {
            uint32_t x = 0, y = 0;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int k = 32 * g + 4 * w + i;
                x |= (uint32_t)a8[r * 128 + k] << (8 * i);
                y |= (uint32_t)b8[k * 16 + r] << (8 * i);
            }
            av[w] = (int)x;
            bv[w] = (int)y;
        }
        // unit block scales (E8M0 127 = 2^0), e4m3 for both operands
        d = __builtin_amdgcn_mfma_scale_f32_16x16x128_f8f6f4(av, bv, c, 0, 0, 0, 127, 0, 127);
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) D[(4 * g + i) * 16 + r] = d[i];
}

}  // namespace

}  // namespace ace

extern "C" ace_status ace_mfma_probe(int32_t kind, const void* A, const void* B, const float* C, float* D,
                                     int32_t device) {
    using namespace ace;
    if (kind < 0 || kind > 2 || !A || !B || !C || !D || device < 0) return ACE_E_INVALID;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device >= ndev) {
        (void)hipGetLastError();
        return ACE_E_DEVICE;
    }
    int prev = -1;
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    if (hipSetDevice(device) != hipSuccess) {
        (void)hipGetLastError();
        return ACE_E_DEVICE;
    }
    const size_t ab = kind == 0 ? 64 * sizeof(float) : kind == 1 ? 512 * sizeof(uint16_t) : 2048;
    void *dA = nullptr, *dB = nullptr;
    float *dC = nullptr, *dD = nullptr;
    hipError_t e = hipMalloc(&dA, ab);
    if (e == hipSuccess) e = hipMalloc(&dB, ab);
    if (e == hipSuccess) e = hipMalloc((void**)&dC, 256 * sizeof(float));
    if (e == hipSuccess) e = hipMalloc((void**)&dD, 256 * sizeof(float));
    if (e == hipSuccess) e = hipMemcpy(dA, A, ab, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(dB, B, ab, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(dC, C, 256 * sizeof(float), hipMemcpyHostToDevice);
    if (e == hipSuccess) {
        if (kind == 0) hipLaunchKernelGGL(mfma_probe_kernel<0>, dim3(1), dim3(64), 0, nullptr, dA, dB, dC, dD);
        else if (kind == 1) hipLaunchKernelGGL(mfma_probe_kernel<1>, dim3(1), dim3(64), 0, nullptr, dA, dB, dC, dD);
        else hipLaunchKernelGGL(mfma_probe_kernel<2>, dim3(1), dim3(64), 0, nullptr, dA, dB, dC, dD);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipMemcpy(D, dD, 256 * sizeof(float), hipMemcpyDeviceToHost);
    void* ptrs[] = {dA, dB, dC, dD};
    for (void* p : ptrs)
        if (p) (void)hipFree(p);
    if (prev >= 0) (void)hipSetDevice(prev);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return ACE_E_DEVICE;
    }
    return ACE_OK;
}
