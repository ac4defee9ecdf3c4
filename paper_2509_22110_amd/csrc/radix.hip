// Stable LSD radix sort of (uint32 key, uint32 value) pairs, digits of 6 to 10 bits.
//
// Per pass: (1) every work-group counts the digits of its 2048-key tile in LDS and writes one
// column of a digit-major histogram; (2) one work-group scans the histogram; (3) every work-group
// re-reads its tile in 8 rounds of 256 keys and writes each key to
// offset[digit][group] + (rank among equal digits before it).  The rank inside a wave comes from
// one ballot per digit bit, across the four waves from LDS counters, so the sort is
// stable and deterministic.
#include "common.hpp"

namespace tpe {

constexpr int RS_THREADS = 256;
constexpr int RS_ROUNDS = 8;
constexpr int RS_TILE = RS_THREADS * RS_ROUNDS;

template <int DB>
__global__ __launch_bounds__(RS_THREADS) void rs_hist(const uint32_t* __restrict__ keys, int64_t n, int shift,
                                                       int nblocks, uint32_t* __restrict__ hist) {
    constexpr int ND = 1 << DB;
    __shared__ uint32_t h[ND];
    const int tid = threadIdx.x;
    for (int d = tid; d < ND; d += RS_THREADS) h[d] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * RS_TILE;
    for (int r = 0; r < RS_ROUNDS; ++r) {
        int64_t i = base + r * RS_THREADS + tid;
        if (i < n) atomicAdd(&h[(keys[i] >> shift) & (ND - 1)], 1u);
    }
    __syncthreads();
    for (int d = tid; d < ND; d += RS_THREADS) hist[(int64_t)d * nblocks + blockIdx.x] = h[d];
}

template <int DB>
__global__ __launch_bounds__(RS_THREADS) void rs_scatter(const uint32_t* __restrict__ kin,
                                                          const uint32_t* __restrict__ vin, int64_t n,
                                                          int shift, int nblocks,
                                                          const uint32_t* __restrict__ off,
                                                          uint32_t* __restrict__ kout,
                                                          uint32_t* __restrict__ vout) {
    constexpr int ND = 1 << DB;
    constexpr int NW = RS_THREADS / 64;
    __shared__ uint32_t run[ND];
    __shared__ uint32_t wcnt[NW][ND];
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    for (int d = tid; d < ND; d += RS_THREADS) {
        run[d] = off[(int64_t)d * nblocks + blockIdx.x];
        for (int w = 0; w < NW; ++w) wcnt[w][d] = 0;
    }
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * RS_TILE;
    const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    for (int r = 0; r < RS_ROUNDS; ++r) {
        const int64_t i = base + r * RS_THREADS + tid;
        const bool act = i < n;
        uint32_t k = act ? kin[i] : 0u;
        uint32_t v = act ? vin[i] : 0u;
        uint32_t d = (k >> shift) & (ND - 1);
        uint64_t peers = __ballot(act);
        for (int b = 0; b < DB; ++b) {
            uint64_t bal = __ballot((d >> b) & 1u);
            peers &= ((d >> b) & 1u) ? bal : ~bal;
        }
        const uint32_t below = (uint32_t)__popcll(peers & lt);
        if (act && below == 0) wcnt[wave][d] = (uint32_t)__popcll(peers);
        __syncthreads();
        if (act) {
            uint32_t pos = run[d] + below;
            for (int w = 0; w < wave; ++w) pos += wcnt[w][d];
            kout[pos] = k;
            vout[pos] = v;
        }
        __syncthreads();
        for (int dd = tid; dd < ND; dd += RS_THREADS) {
            uint32_t add = 0;
            for (int w = 0; w < NW; ++w) { add += wcnt[w][dd]; wcnt[w][dd] = 0; }
            run[dd] += add;
        }
        __syncthreads();
    }
}

// Single-work-group exclusive scan of n counts -> off[0..n] (off[n] = total).
__global__ __launch_bounds__(1024) void exclusive_scan_1wg(const uint32_t* __restrict__ in, int64_t n,
                                                            uint32_t* __restrict__ off) {
    __shared__ uint32_t part[1024];
    const int tid = threadIdx.x;
    const int64_t per = (n + 1023) / 1024;
    const int64_t b = tid * per, e = min(n, b + per);
    uint32_t s = 0;
    for (int64_t i = b; i < e; ++i) s += in[i];
    part[tid] = s;
    __syncthreads();
    for (int o = 1; o < 1024; o <<= 1) {
        uint32_t x = tid >= o ? part[tid - o] : 0u;
        __syncthreads();
        part[tid] += x;
        __syncthreads();
    }
    uint32_t run = part[tid] - s;
    for (int64_t i = b; i < e; ++i) {
        off[i] = run;
        run += in[i];
    }
    if (tid == 1023) off[n] = part[1023];
}

hipError_t launch_exclusive_scan(const uint32_t* in, int64_t n, uint32_t* off, hipStream_t st) {
    hipLaunchKernelGGL(exclusive_scan_1wg, dim3(1), dim3(1024), 0, st, in, n, off);
    return hipGetLastError();
}


// Sorts n pairs by the low `bits` (<= 32) bits of the key in ceil(bits / 10) passes of equal
// digits (<= 10 bits).  Uses (ktmp, vtmp) as ping-pong buffers and hist/off of
// (1024 * ceil(n / RS_TILE) + 1) words.  The result always ends in (keys, vals).
template <int DB>
static hipError_t rs_pass(const uint32_t* ki, const uint32_t* vi, uint32_t* ko, uint32_t* vo, int64_t n, int shift,
                          int nblocks, uint32_t* hist, uint32_t* off, hipStream_t st) {
    hipLaunchKernelGGL((rs_hist<DB>), dim3(nblocks), dim3(RS_THREADS), 0, st, ki, n, shift, nblocks, hist);
    hipLaunchKernelGGL(exclusive_scan_1wg, dim3(1), dim3(1024), 0, st, hist, (int64_t)(1 << DB) * nblocks, off);
    hipLaunchKernelGGL((rs_scatter<DB>), dim3(nblocks), dim3(RS_THREADS), 0, st, ki, vi, n, shift, nblocks, off, ko,
                       vo);
    return hipGetLastError();
}

int64_t radix_hist_words(int64_t n) { return (int64_t)1024 * ((n + RS_TILE - 1) / RS_TILE) + 1; }

hipError_t radix_sort(uint32_t* keys, uint32_t* vals, uint32_t* ktmp, uint32_t* vtmp, int64_t n, int bits,
                      uint32_t* hist, uint32_t* off, hipStream_t st) {
    if (n <= 1 || bits <= 0) return hipSuccess;
    if (bits > 32) bits = 32;
    const int nblocks = (int)((n + RS_TILE - 1) / RS_TILE);
    const int passes = (bits + 9) / 10;
    const int db = (bits + passes - 1) / passes;
    uint32_t *ki = keys, *vi = vals, *ko = ktmp, *vo = vtmp;
    for (int p = 0; p < passes; ++p) {
        hipError_t e;
        switch (db) {
            case 10: e = rs_pass<10>(ki, vi, ko, vo, n, db * p, nblocks, hist, off, st); break;
            case 9: e = rs_pass<9>(ki, vi, ko, vo, n, db * p, nblocks, hist, off, st); break;
            case 8: e = rs_pass<8>(ki, vi, ko, vo, n, db * p, nblocks, hist, off, st); break;
            case 7: e = rs_pass<7>(ki, vi, ko, vo, n, db * p, nblocks, hist, off, st); break;
            default: e = rs_pass<6>(ki, vi, ko, vo, n, db * p, nblocks, hist, off, st); break;
        }
        if (e != hipSuccess) return e;
        std::swap(ki, ko);
        std::swap(vi, vo);
    }
    if (ki != keys) {
        hipError_t e = hipMemcpyAsync(keys, ki, n * sizeof(uint32_t), hipMemcpyDeviceToDevice, st);
        if (e != hipSuccess) return e;
        e = hipMemcpyAsync(vals, vi, n * sizeof(uint32_t), hipMemcpyDeviceToDevice, st);
        if (e != hipSuccess) return e;
    }
    return hipGetLastError();
}

}  // namespace tpe
