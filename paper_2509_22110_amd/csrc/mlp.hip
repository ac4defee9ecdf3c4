// Small MLP for the learned far-field correction: BF16 MFMA (v_mfma_f32_16x16x32_bf16) forward and
// backward with FP32 accumulation, FP32 master weights, Adam.  Not part of the paper: a learned
// correction of the monopole cluster interaction of the Barnes-Hut far field.
//
// Network: x[32] -> relu(W1 x + b1)[64] -> relu(W2 . + b2)[64] -> relu(W3 . + b3)[64] -> W4 . + b4 [16].
// Parameters are stored row-major as W[in][out] followed by b[out], layer after layer (11,472
// floats).  Loss: sum over samples of w_i * sum_{j < 11} (y_ij - t_ij)^2 / (11 * sum_i w_i), where the
// per-sample weight w_i is column 15 of the target row (0 marks an unused row).
//
// MFMA operand layout (16x16x32 bf16, wave64): lane l supplies A[m = l % 16][k = 8 (l / 16) + i] and
// B[k = 8 (l / 16) + i][n = l % 16] for i = 0..7, and receives D[m = 4 (l / 16) + i][n = l % 16] for
// i = 0..3.  Every GEMM below is a sequence of such 16x16x32 steps; operands are gathered element by
// element through small accessor functors, so one routine serves all the transposes of the
// forward and backward passes.
#include <cstdio>
#include <cstring>
#include <random>
#include <vector>

#include "common.hpp"
#include "mlp.hpp"
#include "mlp_infer.hpp"

namespace tpe {

template <int MT, int NT, int KT, class FA, class FB>
__device__ __forceinline__ void wave_gemm(FA a, FB b, f32x4 (&acc)[MT][NT]) {
    const int lane = threadIdx.x & 63;
    const int r = lane & 15, kq = (lane >> 4) * 8;
#pragma unroll
    for (int kt = 0; kt < KT; ++kt) {
        bf16x8 bfr[NT];
#pragma unroll
        for (int nt = 0; nt < NT; ++nt)
#pragma unroll
            for (int i = 0; i < 8; ++i) bfr[nt][i] = (__bf16)b(kt * 32 + kq + i, nt * 16 + r);
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) {
            bf16x8 afr;
#pragma unroll
            for (int i = 0; i < 8; ++i) afr[i] = (__bf16)a(mt * 16 + r, kt * 32 + kq + i);
#pragma unroll
            for (int nt = 0; nt < NT; ++nt)
                acc[mt][nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(afr, bfr[nt], acc[mt][nt], 0, 0, 0);
        }
    }
}

template <int MT, int NT>
__device__ __forceinline__ void zero_acc(f32x4 (&acc)[MT][NT]) {
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) acc[mt][nt] = f32x4{0.f, 0.f, 0.f, 0.f};
}

// Store a D-fragment block to a row-major LDS/global matrix dst[m][n] (leading dimension ld),
// applying f(value, row, col).
template <int MT, int NT, class Fn>
__device__ __forceinline__ void store_acc(const f32x4 (&acc)[MT][NT], float* dst, int ld, Fn f) {
    const int lane = threadIdx.x & 63;
    const int c = lane & 15, r4 = (lane >> 4) * 4;
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
        for (int nt = 0; nt < NT; ++nt)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int row = mt * 16 + r4 + i, col = nt * 16 + c;
                dst[row * ld + col] = f(acc[mt][nt][i], row, col);
            }
}

constexpr int TM = 32;  // samples per training / inference tile (one wave)

// Forward pass of one tile; H1..H3 and Y are LDS [TM][64] / [TM][16] fp32.  Xs: LDS [TM][32].
__device__ void mlp_tile_forward(const float* __restrict__ P, const float* Xs, float* H1, float* H2, float* H3,
                                 float* Y) {
    const float* W1 = P + MLP_OFF_W1;
    const float* b1 = P + MLP_OFF_B1;
    const float* W2 = P + MLP_OFF_W2;
    const float* b2 = P + MLP_OFF_B2;
    const float* W3 = P + MLP_OFF_W3;
    const float* b3 = P + MLP_OFF_B3;
    const float* W4 = P + MLP_OFF_W4;
    const float* b4 = P + MLP_OFF_B4;
    {
        f32x4 acc[TM / 16][4];
        zero_acc(acc);
        wave_gemm<TM / 16, 4, 1>([&](int m, int k) { return Xs[m * 32 + k]; },
                                 [&](int k, int n) { return W1[k * 64 + n]; }, acc);
        store_acc(acc, H1, 64, [&](float v, int, int n) { return fmaxf(v + b1[n], 0.f); });
    }
    __syncthreads();
    {
        f32x4 acc[TM / 16][4];
        zero_acc(acc);
        wave_gemm<TM / 16, 4, 2>([&](int m, int k) { return H1[m * 64 + k]; },
                                 [&](int k, int n) { return W2[k * 64 + n]; }, acc);
        store_acc(acc, H2, 64, [&](float v, int, int n) { return fmaxf(v + b2[n], 0.f); });
    }
    __syncthreads();
    {
        f32x4 acc[TM / 16][4];
        zero_acc(acc);
        wave_gemm<TM / 16, 4, 2>([&](int m, int k) { return H2[m * 64 + k]; },
                                 [&](int k, int n) { return W3[k * 64 + n]; }, acc);
        store_acc(acc, H3, 64, [&](float v, int, int n) { return fmaxf(v + b3[n], 0.f); });
    }
    __syncthreads();
    {
        f32x4 acc[TM / 16][1];
        zero_acc(acc);
        wave_gemm<TM / 16, 1, 2>([&](int m, int k) { return H3[m * 64 + k]; },
                                 [&](int k, int n) { return W4[k * 16 + n]; }, acc);
        store_acc(acc, Y, 16, [&](float v, int, int n) { return v + b4[n]; });
    }
    __syncthreads();
}

// Inference through the routine the far-field walk uses (packed BF16 weights): one wave per 64
// samples, so out[i] is bit-identical to the in-walk prediction for the same features.
__global__ __launch_bounds__(64) void mlp_infer_kernel(const MlpPacked* __restrict__ W, const float* __restrict__ X,
                                                       int64_t n, float* __restrict__ out) {
    __shared__ MlpScratch ms;
    const int64_t row = (int64_t)blockIdx.x * 64 + threadIdx.x;
    float x[32], y[16];
#pragma unroll
    for (int k = 0; k < 32; ++k) x[k] = row < n ? X[row * 32 + k] : 0.f;
    mlp_infer64(W, x, ms, y);
    if (row < n) {
#pragma unroll
        for (int j = 0; j < 16; ++j) out[row * 16 + j] = y[j];
    }
}

// Forward + backward of one tile; writes the tile's parameter gradient (unnormalised sums of
// w * d(sum_j (y - t)^2)) to gpart[tile][MLP_NPARAM] and (sum w (y-t)^2, sum w) to lpart[tile][2].
__global__ __launch_bounds__(64) void mlp_train_tile(const float* __restrict__ P, const float* __restrict__ X,
                                                     const float* __restrict__ T, int64_t n,
                                                     float* __restrict__ gpart, float* __restrict__ lpart, float lam) {
    __shared__ float Xs[TM * 32], H1[TM * 64], H2[TM * 64], H3[TM * 64], D1[TM * 64], D2[TM * 64], Y[TM * 16];
    __shared__ float red[64];
    const int lane = threadIdx.x;
    const int64_t base = (int64_t)blockIdx.x * TM;
    for (int e = lane; e < TM * 32; e += 64) {
        const int64_t row = base + e / 32;
        Xs[e] = row < n ? X[row * 32 + e % 32] : 0.f;
    }
    __syncthreads();
    mlp_tile_forward(P, Xs, H1, H2, H3, Y);
    // dL/dY (up to the global normalisation, applied in the Adam pass) into Y; loss partials.
    // With lam > 0 the loss also compares the differences of neighbouring rows of the tile:
    // lam sum_m w_m w_(m+1) |(y_(m+1) - y_m) - (t_(m+1) - t_m)|^2.
    float ls = 0.f, ws = 0.f;
    for (int e = lane; e < TM * 16; e += 64) {
        const int m = e / 16;
        const int64_t row = base + m;
        const int j = e % 16;
        float g = 0.f;
        if (row < n && j < MLP_NOUT_USED) {
            const float w = T[row * 16 + 15];
            const float d = Y[e] - T[row * 16 + j];
            ls += w * d * d;
            g = 2.f * w * d;
            if (j == 0) ws += w;
            if (lam > 0.f) {
                if (m + 1 < TM && row + 1 < n) {
                    const float v = w * T[(row + 1) * 16 + 15];
                    const float D = (Y[e + 16] - T[(row + 1) * 16 + j]) - d;
                    ls += lam * v * D * D;
                    g -= 2.f * lam * v * D;
                }
                if (m > 0) {
                    const float v = T[(row - 1) * 16 + 15] * w;
                    const float D = d - (Y[e - 16] - T[(row - 1) * 16 + j]);
                    g += 2.f * lam * v * D;
                }
            }
        }
        D1[e] = g;
    }
    __syncthreads();
    for (int e = lane; e < TM * 16; e += 64) Y[e] = D1[e];
    for (int off = 32; off > 0; off >>= 1) {
        ls += __shfl_xor(ls, off);
        ws += __shfl_xor(ws, off);
    }
    if (lane == 0) {
        lpart[2 * blockIdx.x] = ls;
        lpart[2 * blockIdx.x + 1] = ws;
    }
    __syncthreads();
    const float* W2 = P + MLP_OFF_W2;
    const float* W3 = P + MLP_OFF_W3;
    const float* W4 = P + MLP_OFF_W4;
    float* G = gpart + (size_t)blockIdx.x * MLP_NPARAM;
    // layer 4: gW4 = H3^T dY, gb4 = sum dY; dZ3 = (dY W4^T) * (H3 > 0) -> D1
    {
        f32x4 acc[4][1];
        zero_acc(acc);
        wave_gemm<4, 1, 1>([&](int m, int k) { return H3[k * 64 + m]; }, [&](int k, int nn) { return Y[k * 16 + nn]; },
                           acc);
        store_acc(acc, G + MLP_OFF_W4, 16, [](float v, int, int) { return v; });
        for (int c = lane; c < 16; c += 64) {
            float s = 0.f;
            for (int m = 0; m < TM; ++m) s += Y[m * 16 + c];
            G[MLP_OFF_B4 + c] = s;
        }
        f32x4 d[TM / 16][4];
        zero_acc(d);
        wave_gemm<TM / 16, 4, 1>([&](int m, int k) { return k < 16 ? Y[m * 16 + k] : 0.f; },
                                 [&](int k, int nn) { return k < 16 ? W4[nn * 16 + k] : 0.f; }, d);
        store_acc(d, D1, 64, [&](float v, int m, int nn) { return H3[m * 64 + nn] > 0.f ? v : 0.f; });
    }
    __syncthreads();
    // layer 3: gW3 = H2^T dZ3, gb3; dZ2 = (dZ3 W3^T) * (H2 > 0) -> D2
    {
        f32x4 acc[4][4];
        zero_acc(acc);
        wave_gemm<4, 4, 1>([&](int m, int k) { return H2[k * 64 + m]; }, [&](int k, int nn) { return D1[k * 64 + nn]; },
                           acc);
        store_acc(acc, G + MLP_OFF_W3, 64, [](float v, int, int) { return v; });
        for (int c = lane; c < 64; c += 64) {
            float s = 0.f;
            for (int m = 0; m < TM; ++m) s += D1[m * 64 + c];
            G[MLP_OFF_B3 + c] = s;
        }
        f32x4 d[TM / 16][4];
        zero_acc(d);
        wave_gemm<TM / 16, 4, 2>([&](int m, int k) { return D1[m * 64 + k]; },
                                 [&](int k, int nn) { return W3[nn * 64 + k]; }, d);
        store_acc(d, D2, 64, [&](float v, int m, int nn) { return H2[m * 64 + nn] > 0.f ? v : 0.f; });
    }
    __syncthreads();
    // layer 2: gW2 = H1^T dZ2, gb2; dZ1 = (dZ2 W2^T) * (H1 > 0) -> D1
    {
        f32x4 acc[4][4];
        zero_acc(acc);
        wave_gemm<4, 4, 1>([&](int m, int k) { return H1[k * 64 + m]; }, [&](int k, int nn) { return D2[k * 64 + nn]; },
                           acc);
        store_acc(acc, G + MLP_OFF_W2, 64, [](float v, int, int) { return v; });
        for (int c = lane; c < 64; c += 64) {
            float s = 0.f;
            for (int m = 0; m < TM; ++m) s += D2[m * 64 + c];
            G[MLP_OFF_B2 + c] = s;
        }
        __syncthreads();
        f32x4 d[TM / 16][4];
        zero_acc(d);
        wave_gemm<TM / 16, 4, 2>([&](int m, int k) { return D2[m * 64 + k]; },
                                 [&](int k, int nn) { return W2[nn * 64 + k]; }, d);
        store_acc(d, D1, 64, [&](float v, int m, int nn) { return H1[m * 64 + nn] > 0.f ? v : 0.f; });
    }
    __syncthreads();
    // layer 1: gW1 = X^T dZ1, gb1
    {
        f32x4 acc[2][4];
        zero_acc(acc);
        wave_gemm<2, 4, 1>([&](int m, int k) { return Xs[k * 32 + m]; }, [&](int k, int nn) { return D1[k * 64 + nn]; },
                           acc);
        store_acc(acc, G + MLP_OFF_W1, 64, [](float v, int, int) { return v; });
        for (int c = lane; c < 64; c += 64) {
            float s = 0.f;
            for (int m = 0; m < TM; ++m) s += D1[m * 64 + c];
            G[MLP_OFF_B1 + c] = s;
        }
    }
    (void)red;
}

// Sum the tiles' gradients in tile order, normalise by 7 * sum w, Adam-update the FP32 master
// parameters; the last work-group also writes the loss.
__global__ __launch_bounds__(256) void mlp_adam(float* __restrict__ P, float* __restrict__ M, float* __restrict__ Vv,
                                                const float* __restrict__ gpart, const float* __restrict__ lpart,
                                                int ntiles, float lr, float b1t, float b2t, float* __restrict__ loss) {
    __shared__ float wsum_s, lsum_s;
    if (threadIdx.x == 0) {
        float ws = 0.f, ls = 0.f;
        for (int t = 0; t < ntiles; ++t) {
            ls += lpart[2 * t];
            ws += lpart[2 * t + 1];
        }
        wsum_s = ws;
        lsum_s = ls;
    }
    __syncthreads();
    const float norm = wsum_s > 0.f ? 1.f / (MLP_NOUT_USED * wsum_s) : 0.f;
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (blockIdx.x == 0 && threadIdx.x == 0 && loss) loss[0] = lsum_s * norm;
    if (p >= MLP_NPARAM) return;
    float g = 0.f;
    for (int t = 0; t < ntiles; ++t) g += gpart[(size_t)t * MLP_NPARAM + p];
    g *= norm;
    // 1 - beta in FP64 before the rounding to FP32 (1.f - 0.999f is 0.00099998713: 1.3e-5 off)
    const float beta1 = 0.9f, beta2 = 0.999f, eps = 1e-8f;
    const float omb1 = (float)(1.0 - 0.9), omb2 = (float)(1.0 - 0.999);
    const float m = beta1 * M[p] + omb1 * g;
    const float v = beta2 * Vv[p] + omb2 * g * g;
    M[p] = m;
    Vv[p] = v;
    const float mh = m / (1.f - b1t), vh = v / (1.f - b2t);
    P[p] -= lr * mh / (sqrtf(vh) + eps);
}

// Raw (un-normalised, per-sample-weighted) gradient for tests: sum of tile partials.
__global__ void mlp_grad_sum(const float* __restrict__ gpart, const float* __restrict__ lpart, int ntiles,
                             float* __restrict__ grad) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= MLP_NPARAM) return;
    float ws = 0.f;
    for (int t = 0; t < ntiles; ++t) ws += lpart[2 * t + 1];
    const float norm = ws > 0.f ? 1.f / (MLP_NOUT_USED * ws) : 0.f;
    float g = 0.f;
    for (int t = 0; t < ntiles; ++t) g += gpart[(size_t)t * MLP_NPARAM + p];
    grad[p] = g * norm;
}

// FP32 master parameters -> BF16 A fragments in MFMA order + FP32 biases (see mlp_infer.hpp).
__global__ void mlp_pack(const float* __restrict__ P, float min_s, MlpPacked* __restrict__ out) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < MLP_NFRAG * 64) {
        const int f = t / 64, lane = t % 64, r = lane & 15, q = lane >> 4;
        const float* W;
        int ld, kt, mt;
        if (f < 4) { W = P + MLP_OFF_W1; ld = 64; kt = 0; mt = f; }
        else if (f < 12) { W = P + MLP_OFF_W2; ld = 64; kt = (f - 4) / 4; mt = (f - 4) % 4; }
        else if (f < 20) { W = P + MLP_OFF_W3; ld = 64; kt = (f - 12) / 4; mt = (f - 12) % 4; }
        else { W = P + MLP_OFF_W4; ld = 16; kt = f - 20; mt = 0; }
        // A[m = out unit mt * 16 + r][k = in unit kt * 32 + 8 q + i] = W[k][m]
        bf16x8 v;
        for (int i = 0; i < 8; ++i) v[i] = (__bf16)W[(kt * 32 + 8 * q + i) * ld + mt * 16 + r];
        out->frag[f][lane] = v;
    }
    if (t == 0) out->min_s = min_s;
    if (t < 208) {
        float b;
        if (t < 64) b = P[MLP_OFF_B1 + t];
        else if (t < 128) b = P[MLP_OFF_B2 + t - 64];
        else if (t < 192) b = P[MLP_OFF_B3 + t - 128];
        else b = P[MLP_OFF_B4 + t - 192];
        out->bias[t] = b;
    }
}

hipError_t mlp_pack_launch(const float* P, float min_s, void* packed, hipStream_t st) {
    hipLaunchKernelGGL(mlp_pack, dim3((MLP_NFRAG * 64 + 255) / 256), dim3(256), 0, st, P, min_s, (MlpPacked*)packed);
    return hipGetLastError();
}

size_t mlp_packed_bytes() { return sizeof(MlpPacked); }

// ---- host side -------------------------------------------------------------------------------------

void mlp_init_params(uint64_t seed, std::vector<float>& P) {
    // He-uniform weights from a seeded 64-bit Mersenne twister; zero biases
    P.assign(MLP_NPARAM, 0.f);
    std::mt19937_64 g(seed);
    std::uniform_real_distribution<double> U(-1.0, 1.0);
    struct L { int off, in, out; } ls[4] = {{MLP_OFF_W1, 32, 64}, {MLP_OFF_W2, 64, 64}, {MLP_OFF_W3, 64, 64},
                                            {MLP_OFF_W4, 64, 16}};
    for (auto& l : ls) {
        const double bound = std::sqrt(6.0 / l.in);
        for (int i = 0; i < l.in * l.out; ++i) P[l.off + i] = (float)(bound * U(g));
    }
}

hipError_t mlp_infer_launch(const void* packed, const float* X, int64_t n, float* out, hipStream_t st) {
    const int64_t g = (n + 63) / 64;
    if (g == 0) return hipSuccess;
    if (g > 0x7fffffff) return hipErrorInvalidValue;
    hipLaunchKernelGGL(mlp_infer_kernel, dim3((unsigned)g), dim3(64), 0, st, (const MlpPacked*)packed, X, n, out);
    return hipGetLastError();
}

int64_t mlp_tiles(int64_t n) { return (n + TM - 1) / TM; }

hipError_t mlp_train_launch(float* P, float* Mm, float* Vv, const float* X, const float* T, int64_t n, float lr,
                            float lam, int64_t step, float* gpart, float* lpart, float* loss, float* grad_out,
                            hipStream_t st) {
    const int ntiles = (int)mlp_tiles(n);
    hipLaunchKernelGGL(mlp_train_tile, dim3(ntiles), dim3(64), 0, st, P, X, T, n, gpart, lpart, lam);
    if (grad_out) {
        hipLaunchKernelGGL(mlp_grad_sum, dim3((MLP_NPARAM + 255) / 256), dim3(256), 0, st, gpart, lpart, ntiles,
                           grad_out);
        return hipGetLastError();
    }
    const float b1t = (float)std::pow(0.9, (double)step), b2t = (float)std::pow(0.999, (double)step);
    hipLaunchKernelGGL(mlp_adam, dim3((MLP_NPARAM + 255) / 256), dim3(256), 0, st, P, Mm, Vv, gpart, lpart, ntiles, lr,
                       b1t, b2t, loss);
    return hipGetLastError();
}

}  // namespace tpe
