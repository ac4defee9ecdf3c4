// Internal declarations of the far-field MLP (see mlp.hip).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <vector>

namespace tpe {

typedef __attribute__((ext_vector_type(8))) __bf16 bf16x8;
typedef __attribute__((ext_vector_type(4))) float f32x4;

// fixed architecture: 32 -> 64 -> 64 -> 64 -> 16
constexpr int MLP_DIN = 32, MLP_W = 64, MLP_DEPTH = 3, MLP_DOUT = 16;
constexpr int MLP_NOUT_USED = 7;  // outputs that carry a target (K, Sd[3], C[3]; see tree.hip)
constexpr int MLP_OFF_W1 = 0;
constexpr int MLP_OFF_B1 = MLP_OFF_W1 + 32 * 64;
constexpr int MLP_OFF_W2 = MLP_OFF_B1 + 64;
constexpr int MLP_OFF_B2 = MLP_OFF_W2 + 64 * 64;
constexpr int MLP_OFF_W3 = MLP_OFF_B2 + 64;
constexpr int MLP_OFF_B3 = MLP_OFF_W3 + 64 * 64;
constexpr int MLP_OFF_W4 = MLP_OFF_B3 + 64;
constexpr int MLP_OFF_B4 = MLP_OFF_W4 + 64 * 16;
constexpr int MLP_NPARAM = MLP_OFF_B4 + 16;  // 11,472

void mlp_init_params(uint64_t seed, std::vector<float>& P);
hipError_t mlp_infer_launch(const void* packed, const float* X, int64_t n, float* out, hipStream_t st);
int64_t mlp_tiles(int64_t n);
hipError_t mlp_pack_launch(const float* P, float min_s, void* packed, hipStream_t st);
size_t mlp_packed_bytes();
hipError_t mlp_train_launch(float* P, float* Mm, float* Vv, const float* X, const float* T, int64_t n, float lr,
                            float lam, int64_t step, float* gpart, float* lpart, float* loss, float* grad_out,
                            hipStream_t st);

}  // namespace tpe
