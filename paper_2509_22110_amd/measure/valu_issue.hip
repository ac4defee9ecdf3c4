// FP32 VALU issue rate on gfx950: how many cycles one SIMD needs per wave64 instruction for the
// instruction forms and mixes of the pair kernels (a measurement tool, not part of libtpe).
//
// The roofline fractions of the pair kernels are quoted against the published FP32 vector peak,
// 157.3 TFLOP/s = 2 cycles per wave64 FMA per SIMD at 2.4 GHz.  Without packed FP32 (switched off
// for all device code of this project) the question is what the SIMD actually issues; this tool
// measures it for
//   - independent and dependent v_fmac_f32 streams (K chains interleaved round-robin, so an
//     instruction depends on the one K places before it in the same wave),
//   - v_mul_f32, v_add_f32 with a DPP wave rotation (the symmetric kernel's column-sum move),
//     v_rcp_f32 (one per pair),
//   - the two pair mixes: per unordered pair of the symmetric kernel 53 plain FP32 instructions,
//     4 rotations and 1 reciprocal; per ordered pair of the row form 38 plain and 1 reciprocal.
// Every work-group takes 96 KB of LDS, so exactly one of 256 work-groups runs on each of the 256
// CUs and a block of 256 W threads puts W waves on every SIMD.  The kernels touch no memory but
// one store per thread into `out` (256 x 1024 floats).
//
// Build and run (gfx950):
//   hipcc --offload-arch=gfx950 -O3 -Xclang -target-feature -Xclang -packed-fp32-ops \
//         paper_2509_22110_amd/measure/valu_issue.hip -o paper_2509_22110_amd/measure/valu_issue
//   ./paper_2509_22110_amd/measure/valu_issue
// Output: per case, ns per wave64 instruction per SIMD (kernel time / instructions per SIMD) and
// the same in cycles of the clock the SIMDs ran at (measured with the shader cycle counter against
// the 100 MHz constant clock).
#include <hip/hip_runtime.h>
#include <cstdio>

namespace {

constexpr int kLdsBytes = 96 * 1024;
constexpr int kMaxThreads = 1024;

enum Op { FMAC = 0, MUL = 1, DPP = 2, RCP = 3, MIX_SYM = 4, MIX_ROW = 5 };

__device__ __forceinline__ void fmac(float& a, float x, float y) {
    asm volatile("v_fmac_f32 %0, %1, %2" : "+v"(a) : "v"(x), "v"(y));
}
__device__ __forceinline__ void mul(float& a, float y) { asm volatile("v_mul_f32 %0, %0, %1" : "+v"(a) : "v"(y)); }
__device__ __forceinline__ void dpp_rol(float& a, float y) {
    asm volatile("v_add_f32_dpp %0, %0, %1 wave_rol:1 row_mask:0xf bank_mask:0xf bound_ctrl:1" : "+v"(a) : "v"(y));
}
__device__ __forceinline__ void rcp(float& a) { asm volatile("v_rcp_f32 %0, %0" : "+v"(a)); }

// One iteration issues N instructions (N = 24 for the single forms, 58 and 39 for the mixes).
template <int OP, int K>
__global__ __launch_bounds__(kMaxThreads) void issue(float* __restrict__ out, int iters, float s,
                                                    long long* __restrict__ clk) {
    extern __shared__ float lds[];
    float a[12], b[4], r[2];
#pragma unroll
    for (int i = 0; i < 12; ++i) a[i] = threadIdx.x * 1e-3f + i + 1;
#pragma unroll
    for (int i = 0; i < 4; ++i) b[i] = threadIdx.x * 1e-3f + i + 2;
    r[0] = 1.5f + s;
    r[1] = 2.5f + s;
    const float x = s, y = 1.0f - s * 1e-3f;
    const long long c0 = clock64(), w0 = wall_clock64();
    for (int it = 0; it < iters; ++it) {
        if constexpr (OP == FMAC) {
#pragma unroll
            for (int j = 0; j < 24; ++j) fmac(a[j % K], x, y);
        } else if constexpr (OP == MUL) {
#pragma unroll
            for (int j = 0; j < 24; ++j) mul(a[j % K], y);
        } else if constexpr (OP == DPP) {
#pragma unroll
            for (int j = 0; j < 24; ++j) dpp_rol(a[j % K], y);
        } else if constexpr (OP == RCP) {
#pragma unroll
            for (int j = 0; j < 24; ++j) rcp(a[j % K]);
        } else if constexpr (OP == MIX_SYM) {
            // 53 fmac on K chains, a rotation after every 13 of them, one reciprocal in the middle
#pragma unroll
            for (int j = 0; j < 53; ++j) {
                fmac(a[j % K], x, y);
                if (j % 13 == 12) dpp_rol(b[j / 13], y);
                if (j == 26) rcp(r[1]);
            }
        } else if constexpr (OP == MIX_ROW) {
#pragma unroll
            for (int j = 0; j < 38; ++j) {
                fmac(a[j % K], x, y);
                if (j == 19) rcp(r[0]);
            }
        }
    }
    const long long c1 = clock64(), w1 = wall_clock64();
    float acc = r[0] + r[1];
#pragma unroll
    for (int i = 0; i < 12; ++i) acc += a[i];
#pragma unroll
    for (int i = 0; i < 4; ++i) acc += b[i];
    if (s > 1e30f) lds[threadIdx.x] = acc;  // never true: keeps the LDS allocation that sets residency
    out[blockIdx.x * blockDim.x + threadIdx.x] = acc;
    if (blockIdx.x == 0 && threadIdx.x == 0) { clk[0] = c1 - c0; clk[1] = w1 - w0; }
}

int insts_per_iter(int op) { return op == MIX_SYM ? 58 : op == MIX_ROW ? 39 : 24; }

const char* op_name(int op) {
    static const char* n[] = {"fmac", "mul", "add_f32_dpp wave_rol:1", "rcp", "symmetric-kernel mix", "row-form mix"};
    return n[op];
}

template <int OP, int K>
bool run(int w, int iters, float* out, long long* clk) {
    const void* f = reinterpret_cast<const void*>(&issue<OP, K>);
    if (hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, kLdsBytes) != hipSuccess) return false;
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return false;
    hipLaunchKernelGGL((issue<OP, K>), dim3(256), dim3(256 * w), kLdsBytes, 0, out, iters, 0.5f, clk);
    bool ok = hipEventRecord(e0) == hipSuccess;
    hipLaunchKernelGGL((issue<OP, K>), dim3(256), dim3(256 * w), kLdsBytes, 0, out, iters, 0.5f, clk);
    ok = ok && hipGetLastError() == hipSuccess && hipEventRecord(e1) == hipSuccess && hipEventSynchronize(e1) == hipSuccess;
    float ms = 0;
    long long h[2] = {0, 0};
    ok = ok && hipEventElapsedTime(&ms, e0, e1) == hipSuccess &&
         hipMemcpy(h, clk, sizeof(h), hipMemcpyDeviceToHost) == hipSuccess;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (!ok || h[1] <= 0) return false;
    const double ghz = (double)h[0] / ((double)h[1] / 100e6) / 1e9;
    const double ns = ms * 1e6 / ((double)iters * insts_per_iter(OP) * w);
    std::printf("waves/SIMD %d  %-24s K %2d  %.4f ns per wave64 instruction per SIMD = %.2f cycles at %.2f GHz\n",
                w, op_name(OP), K, ns, ns * ghz, ghz);
    std::fflush(stdout);
    return true;
}

}  // namespace

int main() {
    float* out = nullptr;
    long long* clk = nullptr;
    if (hipMalloc(&out, sizeof(float) * 256 * kMaxThreads) != hipSuccess) return 1;
    if (hipMalloc(&clk, sizeof(long long) * 2) != hipSuccess) return 1;
    const int it = 20000;
    bool ok = true;
    for (int w : {2, 3, 4}) {
        ok = ok && run<FMAC, 1>(w, it, out, clk) && run<FMAC, 2>(w, it, out, clk) && run<FMAC, 3>(w, it, out, clk) &&
             run<FMAC, 4>(w, it, out, clk) && run<FMAC, 6>(w, it, out, clk) && run<FMAC, 12>(w, it, out, clk) &&
             run<MUL, 6>(w, it, out, clk) && run<DPP, 6>(w, it, out, clk) && run<RCP, 6>(w, it / 4, out, clk) &&
             run<MIX_SYM, 6>(w, it / 2, out, clk) && run<MIX_ROW, 6>(w, it / 2, out, clk);
    }
    const hipError_t e = hipDeviceSynchronize();
    std::printf("status %s\n", ok && e == hipSuccess ? "ok" : hipGetErrorString(e));
    return ok && e == hipSuccess ? 0 : 1;
}
