// MLP inference for 64 samples held one per lane of a wave (the far-field walk and tpe_mlp_forward
// both call mlp_infer64, so the two give bit-identical results).
//
// Every layer is computed transposed, H_out^T = W^T H_in^T, with v_mfma_f32_16x16x32_bf16:
//   - the weights are the A operand, pre-packed per (layer, k-step, m-tile) so that each lane loads
//     its fragment with one 16-byte load (lane l holds W[k = 8 (l / 16) + i][m = l % 16], i < 8);
//   - the activations are the B operand, read from LDS rows [sample][unit] (BF16) with one 16-byte
//     load per lane (B[k = 8 (l / 16) + i][n = l % 16]);
//   - the accumulators start at the bias, and each lane's D fragment (D[m = 4 (l / 16) + i][n = l %
//     16], i < 4) holds four consecutive units of one sample, so after ReLU and the BF16 conversion it
//     goes back to LDS as one 8-byte store.
// Only LDS traffic of a single wave is involved, which the hardware keeps in program order.  Each
// phase reads what other lanes wrote in the previous one, which the compiler cannot see (to it a
// lane's loads there never alias its own stores), so a compiler memory barrier separates the
// phases: without it a later phase's loads may be scheduled above an earlier phase's stores.
#pragma once
#include "mlp.hpp"

namespace tpe {

typedef __attribute__((ext_vector_type(4))) __bf16 bf16x4;

// A fragments of the four layers: layer 1 (K 32, M 64): 4 fragments [mt]; layers 2 and 3 (K 64,
// M 64): 8 each [kt][mt]; layer 4 (K 64, M 16): 2 [kt].  Biases b1, b2, b3 (64 each) then b4 (16).
constexpr int MLP_NFRAG = 22;
struct MlpPacked {
    bf16x8 frag[MLP_NFRAG][64];
    float bias[208];
    float min_s;  // the correction is applied to far clusters with r_B / rho >= min_s only
    float pad[3];
};

// LDS row strides, padded so that the 16 rows one fragment load touches fall in different banks
constexpr int MLP_XS = 40;  // 32 features (bf16)
constexpr int MLP_HS = 72;  // 64 hidden units (bf16)
constexpr int MLP_YS = 20;  // 16 outputs (float)

// One region for the features, the hidden activations and the outputs: every layer issues all
// its loads before its first store (and a wave's LDS accesses run in order), so each layer may
// overwrite its own input, as layers 2 and 3 do in place.
union MlpScratch {
    __bf16 h[64 * MLP_HS];   // hidden activations
    __bf16 xs[64 * MLP_XS];  // features (layer 1's input)
    float ys[64 * MLP_YS];   // outputs (layer 4's)
};

// BF16 conversion, then the ReLU as a packed 16-bit integer max on the bit patterns (a negative
// BF16 value is a negative int16, and rounding keeps the sign): two values per v_pk_max_i16,
// where fmaxf before the conversion needs two maxes per value (one to canonicalise NaNs).
typedef __attribute__((ext_vector_type(2))) float f32x2;
typedef __attribute__((ext_vector_type(2))) __bf16 bf16x2;
typedef __attribute__((ext_vector_type(2))) short s16x2;
__device__ __forceinline__ uint32_t relu_pk(float a, float b) {
    const s16x2 v = __builtin_bit_cast(s16x2, __builtin_convertvector(f32x2{a, b}, bf16x2));
    return __builtin_bit_cast(uint32_t, __builtin_elementwise_max(v, s16x2{0, 0}));
}
// the four values of a D fragment, as four BF16 values in 8 bytes
__device__ __forceinline__ uint2 relu_bf16x4(f32x4 v) { return make_uint2(relu_pk(v.x, v.y), relu_pk(v.z, v.w)); }

// the packed weights, read through an explicitly global pointer (global_load, not flat)
typedef const __attribute__((address_space(1))) MlpPacked GlobalMlp;
typedef const __attribute__((address_space(1))) f32x4 GlobalF32x4;

// compiler memory barrier between the LDS phases of a wave (see the top of this file)
__device__ __forceinline__ void lds_phase() { asm volatile("" ::: "memory"); }

// One hidden layer: dst[sample][0..64) = relu(W^T src + b), K = 32 * KT.  dst may be src: every
// load of src is issued before the first store.  The bias is the C operand of the first k-step.
template <int KT>
__device__ __forceinline__ void mlp_hidden(GlobalMlp* __restrict__ W, int f0, int boff, const __bf16* src,
                                           int sstride, __bf16* dst) {
    const int lane = threadIdx.x & 63, r = lane & 15, q = lane >> 4;
    f32x4 acc[4][4];
#pragma unroll
    for (int kt = 0; kt < KT; ++kt) {
        bf16x8 bfr[4];
#pragma unroll
        for (int nt = 0; nt < 4; ++nt)
            bfr[nt] = *reinterpret_cast<const bf16x8*>(src + (nt * 16 + r) * sstride + kt * 32 + 8 * q);
#pragma unroll
        for (int mt = 0; mt < 4; ++mt) {
            const bf16x8 a = W->frag[f0 + kt * 4 + mt][lane];
            const f32x4 b = kt == 0 ? *reinterpret_cast<GlobalF32x4*>(W->bias + boff + mt * 16 + 4 * q)
                                    : f32x4{};
#pragma unroll
            for (int nt = 0; nt < 4; ++nt)
                acc[mt][nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, bfr[nt], kt == 0 ? b : acc[mt][nt], 0, 0, 0);
        }
    }
    lds_phase();  // no store moves above a load of src (dst overlaps it)
#pragma unroll
    for (int mt = 0; mt < 4; ++mt)
#pragma unroll
        for (int nt = 0; nt < 4; ++nt)
            *reinterpret_cast<uint2*>(dst + (nt * 16 + r) * MLP_HS + mt * 16 + 4 * q) = relu_bf16x4(acc[mt][nt]);
}


// y = MLP(x) for the wave's 64 samples (lane = sample).
__device__ __forceinline__ void mlp_infer64(const MlpPacked* __restrict__ W, const float (&x)[32], MlpScratch& s,
                                            float (&y)[16]) {
    const int lane = threadIdx.x & 63, r = lane & 15, q = lane >> 4;
    lds_phase();  // the previous call's reads of the scratch come first
    // Reload the weights (cache-resident, 23 KB) on every call instead of letting the compiler keep
    // all fragments and biases in registers across the caller's loop, which would cost occupancy.
    asm volatile("" : "+s"(W));
    GlobalMlp* Wg = (GlobalMlp*)W;  // generic -> global address space
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        f32x4 lo = {x[8 * j], x[8 * j + 1], x[8 * j + 2], x[8 * j + 3]};
        f32x4 hi = {x[8 * j + 4], x[8 * j + 5], x[8 * j + 6], x[8 * j + 7]};
        const bf16x4 l4 = __builtin_convertvector(lo, bf16x4), h4 = __builtin_convertvector(hi, bf16x4);
        *reinterpret_cast<bf16x8*>(s.xs + lane * MLP_XS + 8 * j) = bf16x8{l4.x, l4.y, l4.z, l4.w, h4.x, h4.y, h4.z, h4.w};
    }
    lds_phase();
    mlp_hidden<1>(Wg, 0, 0, s.xs, MLP_XS, s.h);
    lds_phase();
    mlp_hidden<2>(Wg, 4, 64, s.h, MLP_HS, s.h);
    lds_phase();
    mlp_hidden<2>(Wg, 12, 128, s.h, MLP_HS, s.h);
    lds_phase();
    // output layer (linear, M 16)
    f32x4 o[4];
    const f32x4 b = *reinterpret_cast<GlobalF32x4*>(Wg->bias + 192 + 4 * q);
#pragma unroll
    for (int kt = 0; kt < 2; ++kt) {
        const bf16x8 a = Wg->frag[20 + kt][lane];
#pragma unroll
        for (int nt = 0; nt < 4; ++nt) {
            const bf16x8 bf = *reinterpret_cast<const bf16x8*>(s.h + (nt * 16 + r) * MLP_HS + kt * 32 + 8 * q);
            o[nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, bf, kt == 0 ? b : o[nt], 0, 0, 0);
        }
    }
    lds_phase();  // the outputs overlap the activations: every load first (float and bf16 stores
                  // would otherwise count as unrelated to the bf16 loads)
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) *reinterpret_cast<f32x4*>(s.ys + (nt * 16 + r) * MLP_YS + 4 * q) = o[nt];
    lds_phase();
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const f32x4 v = *reinterpret_cast<const f32x4*>(s.ys + lane * MLP_YS + 4 * j);
        y[4 * j] = v.x;
        y[4 * j + 1] = v.y;
        y[4 * j + 2] = v.z;
        y[4 * j + 3] = v.w;
    }
}

}  // namespace tpe
