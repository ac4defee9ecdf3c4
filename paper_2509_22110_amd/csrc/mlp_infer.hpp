// MLP inference for 64 samples held one per lane of a wave (used inside the far-field walk).
// Weights come pre-packed in MFMA B-fragment order (one 16-byte load per lane per fragment);
// activations pass between layers through LDS as BF16, row-major [sample][unit].
#pragma once
#include "mlp.hpp"

namespace tpe {

// B fragments of the four layers: layer 1 (K 32, N 64): 4 fragments [nt]; layer 2 and 3 (K 64,
// N 64): 8 each [kt][nt]; layer 4 (K 64, N 16): 2 [kt].  Biases b1, b2, b3 (64 each) then b4 (16).
constexpr int MLP_NFRAG = 22;
struct MlpPacked {
    bf16x8 frag[MLP_NFRAG][64];
    float bias[208];
    float min_s;  // the correction is applied to far clusters with r_B / rho >= min_s only
    float pad[3];
};

struct MlpScratch {
    __bf16 xs[64 * 32];
    __bf16 ha[64 * 64];
    __bf16 hb[64 * 64];
    float ys[64 * 16];
};

template <int NT>
__device__ __forceinline__ void relu_store_bf16(const f32x4 (&acc)[4][NT], const float* __restrict__ bias,
                                                __bf16* dst) {
    const int lane = threadIdx.x & 63, r = lane & 15, q = lane >> 4;
#pragma unroll
    for (int mt = 0; mt < 4; ++mt)
#pragma unroll
        for (int nt = 0; nt < NT; ++nt)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int row = mt * 16 + 4 * q + i, col = nt * 16 + r;
                dst[row * 64 + col] = (__bf16)fmaxf(acc[mt][nt][i] + bias[col], 0.f);
            }
}

__device__ __forceinline__ void mlp_infer64(const MlpPacked* __restrict__ W, const float (&x)[32], MlpScratch& s,
                                            float (&y)[16]) {
    const int lane = threadIdx.x & 63, r = lane & 15, q = lane >> 4;
#pragma unroll
    for (int k = 0; k < 32; ++k) s.xs[lane * 32 + k] = (__bf16)x[k];
    f32x4 acc[4][4];
    // layer 1
#pragma unroll
    for (int mt = 0; mt < 4; ++mt)
#pragma unroll
        for (int nt = 0; nt < 4; ++nt) acc[mt][nt] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int mt = 0; mt < 4; ++mt) {
        const bf16x8 a = *reinterpret_cast<const bf16x8*>(&s.xs[(mt * 16 + r) * 32 + 8 * q]);
#pragma unroll
        for (int nt = 0; nt < 4; ++nt)
            acc[mt][nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, W->frag[nt][lane], acc[mt][nt], 0, 0, 0);
    }
    relu_store_bf16<4>(acc, W->bias, s.ha);
    // layers 2 and 3
#pragma unroll
    for (int layer = 0; layer < 2; ++layer) {
        const __bf16* src = layer == 0 ? s.ha : s.hb;
        __bf16* dst = layer == 0 ? s.hb : s.ha;
        const int f0 = 4 + 8 * layer;
#pragma unroll
        for (int mt = 0; mt < 4; ++mt)
#pragma unroll
            for (int nt = 0; nt < 4; ++nt) acc[mt][nt] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int kt = 0; kt < 2; ++kt)
#pragma unroll
            for (int mt = 0; mt < 4; ++mt) {
                const bf16x8 a = *reinterpret_cast<const bf16x8*>(&src[(mt * 16 + r) * 64 + kt * 32 + 8 * q]);
#pragma unroll
                for (int nt = 0; nt < 4; ++nt)
                    acc[mt][nt] =
                        __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, W->frag[f0 + kt * 4 + nt][lane], acc[mt][nt], 0, 0, 0);
            }
        relu_store_bf16<4>(acc, W->bias + 64 * (layer + 1), dst);
    }
    // layer 4 (linear)
    f32x4 o[4];
#pragma unroll
    for (int mt = 0; mt < 4; ++mt) o[mt] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int kt = 0; kt < 2; ++kt)
#pragma unroll
        for (int mt = 0; mt < 4; ++mt) {
            const bf16x8 a = *reinterpret_cast<const bf16x8*>(&s.ha[(mt * 16 + r) * 64 + kt * 32 + 8 * q]);
            o[mt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, W->frag[20 + kt][lane], o[mt], 0, 0, 0);
        }
#pragma unroll
    for (int mt = 0; mt < 4; ++mt)
#pragma unroll
        for (int i = 0; i < 4; ++i) s.ys[(mt * 16 + 4 * q + i) * 16 + r] = o[mt][i] + W->bias[192 + r];
#pragma unroll
    for (int j = 0; j < 16; ++j) y[j] = s.ys[lane * 16 + j];
}

}  // namespace tpe
