// Stable LSD radix sort of (uint32 key, uint32 value) pairs, digits of 6 to 10 bits.
//
// Per pass: (1) every work-group counts the digits of its 2048-key tile in LDS and writes one
// column of a digit-major histogram; (2) one work-group scans the histogram; (3) every work-group
// re-reads its tile, each wave a contiguous quarter in 8 rounds of 64 keys, and writes each key to
// offset[digit][group] + (equal digits of lower waves) + (rank among equal digits before it in
// the wave).  The rank inside a round comes from one ballot per digit bit, so the sort is stable
// and deterministic.
#include "common.hpp"

namespace tpe {

constexpr int RS_THREADS = 256;
constexpr int RS_ROUNDS = 8;
constexpr int RS_TILE = RS_THREADS * RS_ROUNDS;

template <int DB>
__global__ __launch_bounds__(RS_THREADS) void rs_hist(const uint32_t* __restrict__ keys, int64_t n, uint32_t kmask,
                                                       int shift, int nblocks, uint32_t* __restrict__ hist) {
    constexpr int ND = 1 << DB;
    __shared__ uint32_t h[ND];
    const int tid = threadIdx.x;
    for (int d = tid; d < ND; d += RS_THREADS) h[d] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * RS_TILE;
    uint32_t kr[RS_ROUNDS];
#pragma unroll
    for (int r = 0; r < RS_ROUNDS; ++r) {
        const int64_t i = base + r * RS_THREADS + tid;
        kr[r] = i < n ? keys[i] : 0u;
    }
#pragma unroll
    for (int r = 0; r < RS_ROUNDS; ++r) {
        const int64_t i = base + r * RS_THREADS + tid;
        if (i < n) atomicAdd(&h[((kr[r] & kmask) >> shift) & (ND - 1)], 1u);
    }
    __syncthreads();
    for (int d = tid; d < ND; d += RS_THREADS) hist[(int64_t)d * nblocks + blockIdx.x] = h[d];
}

// Up to RS_FUSE_BLOCKS tiles the scatter work-groups compute their offsets from the histogram
// themselves (no scan launch): the offset of (digit d, tile b) is the count of all smaller digits
// plus the count of digit d in tiles before b.
constexpr int RS_FUSE_BLOCKS = 64;

__device__ __forceinline__ uint32_t rs_wave_inclusive_scan(uint32_t v) {
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t u = __shfl_up(v, o, 64);
        if (lane >= o) v += u;
    }
    return v;
}

// Wave w of the work-group owns the WR rounds of 64 consecutive keys starting at tile offset
// w * WR * 64; equal digits keep their input order: wave, then round, then lane.  FUSED: `off`
// is the histogram itself (digit-major, nblocks <= RS_FUSE_BLOCKS), else its exclusive scan.
template <int DB, bool FUSED>
__global__ __launch_bounds__(RS_THREADS) void rs_scatter(const uint32_t* __restrict__ kin,
                                                          const uint32_t* __restrict__ vin, int64_t n,
                                                          uint32_t kmask, int shift, int nblocks,
                                                          const uint32_t* __restrict__ off,
                                                          uint32_t* __restrict__ kout,
                                                          uint32_t* __restrict__ vout) {
    constexpr int ND = 1 << DB;
    constexpr int NW = RS_THREADS / 64;
    constexpr int WR = RS_TILE / RS_THREADS;  // rounds per wave
    __shared__ uint32_t pos[NW][ND];          // (wave, digit): count, then running position
    __shared__ uint32_t boff[FUSED ? ND : 1];  // FUSED: this tile's offset of each digit
    __shared__ uint32_t wsum[NW];
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    if constexpr (FUSED) {
        // thread t takes digits [t DPT, (t + 1) DPT): their totals and this tile's prefix
        constexpr int DPT = (ND + RS_THREADS - 1) / RS_THREADS;
        uint32_t tot[DPT], pre[DPT], sum = 0;
#pragma unroll
        for (int j = 0; j < DPT; ++j) {
            const int d = tid * DPT + j;
            tot[j] = pre[j] = 0;
            if (d < ND)
                for (int b = 0; b < nblocks; ++b) {
                    const uint32_t c = off[(int64_t)d * nblocks + b];
                    tot[j] += c;
                    pre[j] += b < (int)blockIdx.x ? c : 0u;
                }
            sum += tot[j];
        }
        const uint32_t inc = rs_wave_inclusive_scan(sum);
        if (lane == 63) wsum[wave] = inc;
        __syncthreads();
        uint32_t run = inc - sum;
        for (int w = 0; w < wave; ++w) run += wsum[w];
#pragma unroll
        for (int j = 0; j < DPT; ++j) {
            const int d = tid * DPT + j;
            if (d < ND) boff[d] = run + pre[j];
            run += tot[j];
        }
    }
    for (int e = tid; e < NW * ND; e += RS_THREADS) pos[e / ND][e % ND] = 0;
    __syncthreads();
    const int64_t wbase = (int64_t)blockIdx.x * RS_TILE + (int64_t)wave * WR * 64;
    uint32_t kr[WR], vr[WR];
#pragma unroll
    for (int r = 0; r < WR; ++r) {
        const int64_t i = wbase + r * 64 + lane;
        kr[r] = i < n ? kin[i] : 0u;
        vr[r] = i < n ? vin[i] : 0u;
    }
#pragma unroll
    for (int r = 0; r < WR; ++r)
        if (wbase + r * 64 + lane < n) atomicAdd(&pos[wave][((kr[r] & kmask) >> shift) & (ND - 1)], 1u);
    __syncthreads();
    for (int d = tid; d < ND; d += RS_THREADS) {
        uint32_t run = FUSED ? boff[d] : off[(int64_t)d * nblocks + blockIdx.x];
        for (int w = 0; w < NW; ++w) {
            const uint32_t c = pos[w][d];
            pos[w][d] = run;
            run += c;
        }
    }
    __syncthreads();
    const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
#pragma unroll
    for (int r = 0; r < WR; ++r) {
        const bool act = wbase + r * 64 + lane < n;
        const uint32_t d = ((kr[r] & kmask) >> shift) & (ND - 1);
        uint64_t peers = __ballot(act);
#pragma unroll
        for (int b = 0; b < DB; ++b) {
            const uint64_t bal = __ballot((d >> b) & 1u);
            peers &= ((d >> b) & 1u) ? bal : ~bal;
        }
        const uint32_t below = (uint32_t)__popcll(peers & lt);
        uint32_t* slot = &pos[wave][d];
        const uint32_t p = *slot + below;
        if (act) {
            kout[p] = kr[r];
            vout[p] = vr[r];
        }
        __builtin_amdgcn_wave_barrier();  // every lane has read its position before it moves
        if (act && below == 0) *slot += (uint32_t)__popcll(peers);
        __builtin_amdgcn_wave_barrier();
    }
}

// Exclusive scan of n counts -> off[0..n] (off[n] = total), in tiles of SCAN_TILE counts.
// Each tile is read and written coalesced through LDS; a thread scans 16 consecutive counts, the
// 1024 thread totals are scanned across the work-group with wave shuffles.  Up to SCAN_SMALL_TILES
// tiles one work-group walks the tiles with a running carry (one launch); above, (1) every
// work-group reduces its tile, (2) one work-group scans the tile sums, (3) every work-group scans
// its tile from its tile's offset.
constexpr int SCAN_T = 1024;
constexpr int SCAN_PER = 16;
constexpr int SCAN_TILE = SCAN_T * SCAN_PER;
constexpr int SCAN_SMALL_TILES = 2;

// thread t's row starts at (SCAN_PER + 1) t: an odd stride, free of bank conflicts
__device__ __forceinline__ int scan_pad(int i) { return i + i / SCAN_PER; }

__device__ __forceinline__ uint32_t wave_inclusive_scan(uint32_t v) {
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t u = __shfl_up(v, o, 64);
        if (lane >= o) v += u;
    }
    return v;
}

// Work-group exclusive scan of one value per thread; *total <- the sum (all threads).
__device__ __forceinline__ uint32_t block_exclusive_scan(uint32_t v, uint32_t* wsum, uint32_t* total) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const uint32_t inc = wave_inclusive_scan(v);
    if (lane == 63) wsum[wave] = inc;
    __syncthreads();
    uint32_t before = 0, all = 0;
#pragma unroll
    for (int w = 0; w < SCAN_T / 64; ++w) {
        const uint32_t x = wsum[w];
        before += w < wave ? x : 0u;
        all += x;
    }
    __syncthreads();
    *total = all;
    return before + inc - v;
}

__global__ __launch_bounds__(SCAN_T) void scan_reduce(const uint32_t* __restrict__ in, int64_t n,
                                                      uint32_t* __restrict__ sums) {
    __shared__ uint32_t wsum[SCAN_T / 64];
    const int64_t base = (int64_t)blockIdx.x * SCAN_TILE;
    uint32_t s = 0;
#pragma unroll
    for (int j = 0; j < SCAN_PER; ++j) {
        const int64_t i = base + j * SCAN_T + threadIdx.x;
        if (i < n) s += in[i];
    }
    uint32_t total;
    (void)block_exclusive_scan(s, wsum, &total);
    if (threadIdx.x == 0) sums[blockIdx.x] = total;
}

// Work-group b scans tiles [b * tpb, min((b + 1) * tpb, ntiles)) starting from boff[b] (0 if
// boff is null); the work-group holding the last tile writes off[n].
__global__ __launch_bounds__(SCAN_T) void scan_tiles(const uint32_t* __restrict__ in, int64_t n,
                                                     const uint32_t* __restrict__ boff, int tpb,
                                                     uint32_t* __restrict__ off) {
    __shared__ uint32_t tile[SCAN_TILE + SCAN_TILE / SCAN_PER];
    __shared__ uint32_t wsum[SCAN_T / 64];
    const int t = threadIdx.x;
    const int64_t ntiles = (n + SCAN_TILE - 1) / SCAN_TILE;
    uint32_t carry = boff ? boff[blockIdx.x] : 0u;
    const int64_t t0 = (int64_t)blockIdx.x * tpb, t1 = t0 + tpb < ntiles ? t0 + tpb : ntiles;
    for (int64_t tb = t0; tb < t1; ++tb) {
        const int64_t base = tb * SCAN_TILE;
#pragma unroll
        for (int j = 0; j < SCAN_PER; ++j) {
            const int64_t i = base + j * SCAN_T + t;
            tile[scan_pad(j * SCAN_T + t)] = i < n ? in[i] : 0u;
        }
        __syncthreads();
        uint32_t v[SCAN_PER], s = 0;
#pragma unroll
        for (int k = 0; k < SCAN_PER; ++k) {
            v[k] = tile[scan_pad(t * SCAN_PER + k)];
            s += v[k];
        }
        uint32_t total;
        uint32_t run = carry + block_exclusive_scan(s, wsum, &total);
#pragma unroll
        for (int k = 0; k < SCAN_PER; ++k) {
            tile[scan_pad(t * SCAN_PER + k)] = run;
            run += v[k];
        }
        __syncthreads();
#pragma unroll
        for (int j = 0; j < SCAN_PER; ++j) {
            const int64_t i = base + j * SCAN_T + t;
            if (i < n) off[i] = tile[scan_pad(j * SCAN_T + t)];
        }
        __syncthreads();
        carry += total;
    }
    if (t == 0 && t1 == ntiles && t0 < t1) off[n] = carry;
    if (t == 0 && ntiles == 0 && blockIdx.x == 0) off[0] = carry;
}

// Single-work-group exclusive scan of a short array (the tile sums).
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

int64_t scan_ws_words(int64_t n) {
    const int64_t nt = (n + SCAN_TILE - 1) / SCAN_TILE;
    return nt <= SCAN_SMALL_TILES ? 0 : 2 * (nt + 1) + 64;
}

hipError_t launch_exclusive_scan(const uint32_t* in, int64_t n, uint32_t* off, uint32_t* ws, hipStream_t st) {
    const int64_t nt = (n + SCAN_TILE - 1) / SCAN_TILE;
    if (nt <= SCAN_SMALL_TILES) {
        hipLaunchKernelGGL(scan_tiles, dim3(1), dim3(SCAN_T), 0, st, in, n, (const uint32_t*)nullptr,
                           (int)(nt > 0 ? nt : 1), off);
        return hipGetLastError();
    }
    if (nt > 0x7fffffff || !ws) return hipErrorInvalidValue;
    uint32_t* sums = ws;
    uint32_t* soff = ws + nt + 1;
    hipLaunchKernelGGL(scan_reduce, dim3((unsigned)nt), dim3(SCAN_T), 0, st, in, n, sums);
    hipLaunchKernelGGL(exclusive_scan_1wg, dim3(1), dim3(1024), 0, st, sums, nt, soff);
    hipLaunchKernelGGL(scan_tiles, dim3((unsigned)nt), dim3(SCAN_T), 0, st, in, n, soff, 1, off);
    return hipGetLastError();
}

// Stable sort of n pairs by the low `bits` (<= 32) bits of the key in ceil(bits / 10) passes of
// equal digits (<= 10 bits), three launches each (two up to RS_FUSE_BLOCKS tiles).  Uses (ktmp, vtmp) as ping-pong buffers and hist/off of
// radix_hist_words(n) words (the histogram, its scan, and the scan's workspace at the end of off).
// The result always ends in (keys, vals).
template <int DB>
static hipError_t rs_pass(const uint32_t* ki, const uint32_t* vi, uint32_t* ko, uint32_t* vo, int64_t n,
                          uint32_t kmask, int shift, int nblocks, uint32_t* hist, uint32_t* off, hipStream_t st) {
    hipLaunchKernelGGL((rs_hist<DB>), dim3(nblocks), dim3(RS_THREADS), 0, st, ki, n, kmask, shift, nblocks, hist);
    if (nblocks <= RS_FUSE_BLOCKS) {
        hipLaunchKernelGGL((rs_scatter<DB, true>), dim3(nblocks), dim3(RS_THREADS), 0, st, ki, vi, n, kmask, shift,
                           nblocks, hist, ko, vo);
        return hipGetLastError();
    }
    const int64_t m = (int64_t)(1 << DB) * nblocks;
    hipError_t e = launch_exclusive_scan(hist, m, off, off + (int64_t)1024 * nblocks + 1, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((rs_scatter<DB, false>), dim3(nblocks), dim3(RS_THREADS), 0, st, ki, vi, n, kmask, shift,
                       nblocks, off, ko, vo);
    return hipGetLastError();
}

int64_t radix_hist_words(int64_t n) {
    const int64_t m = (int64_t)1024 * ((n + RS_TILE - 1) / RS_TILE);
    return m + 1 + scan_ws_words(m);
}

hipError_t radix_sort(uint32_t* keys, uint32_t* vals, uint32_t* ktmp, uint32_t* vtmp, int64_t n, int bits,
                      uint32_t* hist, uint32_t* off, hipStream_t st) {
    if (n <= 1 || bits <= 0) return hipSuccess;
    if (bits > 32) bits = 32;
    // digits are taken from the low `bits` bits only (a pass's digit may reach above them)
    const uint32_t kmask = bits >= 32 ? 0xffffffffu : (1u << bits) - 1u;
    const int nblocks = (int)((n + RS_TILE - 1) / RS_TILE);
    const int passes = (bits + 9) / 10;
    const int db = (bits + passes - 1) / passes;
    uint32_t *ki = keys, *vi = vals, *ko = ktmp, *vo = vtmp;
    for (int p = 0; p < passes; ++p) {
        hipError_t e;
        switch (db) {
            case 10: e = rs_pass<10>(ki, vi, ko, vo, n, kmask, db * p, nblocks, hist, off, st); break;
            case 9: e = rs_pass<9>(ki, vi, ko, vo, n, kmask, db * p, nblocks, hist, off, st); break;
            case 8: e = rs_pass<8>(ki, vi, ko, vo, n, kmask, db * p, nblocks, hist, off, st); break;
            case 7: e = rs_pass<7>(ki, vi, ko, vo, n, kmask, db * p, nblocks, hist, off, st); break;
            default: e = rs_pass<6>(ki, vi, ko, vo, n, kmask, db * p, nblocks, hist, off, st); break;
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
