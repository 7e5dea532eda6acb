// Tile binning and depth sort (GS^3LAM Sec. 3.2.1: the tile-based rasterizer
// of the cited 3DGS work sorts Gaussians in depth order per tile).
//
// Two stable sorts replace one wide-key sort:
//   1. the visible (view, Gaussian) pairs, compacted in (view, index) order,
//      are radix-sorted by the binary32 bits of their camera depth (4 passes
//      of 8 bits);
//   2. each pair, in that depth order, emits one instance per tile of its
//      rectangle, keyed by global tile id, and the instances are radix-sorted
//      by tile id (ceil(log2 tiles) bits).
// Because both sorts are stable and the compaction preserves the index order,
// the final order is (view, tile, depth bits, Gaussian index).
//
// Every count that the host does not know (visible pairs, instances) stays on
// the device; grids are sized for the capacity and blocks beyond the count
// exit early, so the whole pipeline is graph-capturable.
#include "sgs_common.h"

namespace sgs {

namespace {

constexpr int SCAN_THREADS = 256;
constexpr int SCAN_ITEMS = 8;
constexpr int SCAN_TILE = SCAN_THREADS * SCAN_ITEMS;
constexpr int TOP_THREADS = 1024;

// Radix passes run on a fixed grid of at most RS_MAXBLK blocks; the device
// side count is split into contiguous chunks (multiples of RS_THREADS), one
// per block, so the digit histograms stay small whatever the capacity and
// only blocks with elements do work.
constexpr int RS_THREADS = 256;
constexpr int RS_MAXBLK = 1024;
constexpr int RS_WAVES = RS_THREADS / kWave;

int rs_blocks(int64_t n_max) {
    const int64_t b = (n_max + RS_THREADS - 1) / RS_THREADS;
    return (int)(b < RS_MAXBLK ? (b > 0 ? b : 1) : RS_MAXBLK);
}

__device__ __forceinline__ void rs_chunk(int64_t count, int nblk, int64_t& lo, int64_t& hi) {
    const int64_t per = ((count + nblk - 1) / nblk + RS_THREADS - 1) / RS_THREADS * RS_THREADS;
    lo = (int64_t)blockIdx.x * per;
    lo = lo < count ? lo : count;
    hi = lo + per < count ? lo + per : count;
}

__device__ __forceinline__ int64_t eff_count(const int64_t* count_dev, int64_t n_max) {
    if (count_dev == nullptr) return n_max;
    const int64_t c = *count_dev;
    return c < n_max ? c : n_max;
}

// ----------------------------------------------------------------------------
// loaders for the generic exclusive scan
// ----------------------------------------------------------------------------
struct LoadNonZero {  // 1 if touched[i] > 0
    const int32_t* p;
    __device__ uint32_t operator()(int64_t i) const { return p[i] > 0 ? 1u : 0u; }
};
struct LoadGatherTouched {  // touched[idx[i]]
    const int32_t* touched;
    const uint32_t* idx;
    __device__ uint32_t operator()(int64_t i) const { return (uint32_t)touched[idx[i]]; }
};
struct LoadU32 {
    const uint32_t* p;
    __device__ uint32_t operator()(int64_t i) const { return p[i]; }
};

// Exclusive scan of the block's NT thread totals (wave scans, then the wave
// totals in LDS); *total receives the block total.
template <int NT>
__device__ uint32_t block_exclusive(uint32_t v, uint32_t* s_tmp, uint32_t* total) {
    const int tid = threadIdx.x, lane = tid & (kWave - 1), wave = tid / kWave;
    uint32_t x = v;
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        uint32_t y = __shfl_up(x, d, kWave);
        if (lane >= d) x += y;
    }
    if (lane == kWave - 1) s_tmp[wave] = x;
    __syncthreads();
    uint32_t wbase = 0, tot = 0;
    for (int w = 0; w < NT / kWave; ++w) {
        const uint32_t s = s_tmp[w];
        if (w < wave) wbase += s;
        tot += s;
    }
    __syncthreads();
    *total = tot;
    return wbase + x - v;
}

template <class Load>
__global__ void __launch_bounds__(SCAN_THREADS) k_scan_partial(Load ld, const int64_t* count_dev, int64_t n_max,
                                                               uint32_t* block_sums) {
    __shared__ uint32_t s_tmp[SCAN_THREADS / kWave];
    const int64_t count = eff_count(count_dev, n_max);
    const int64_t base = (int64_t)blockIdx.x * SCAN_TILE + (int64_t)threadIdx.x * SCAN_ITEMS;
    uint32_t acc = 0;
#pragma unroll
    for (int k = 0; k < SCAN_ITEMS; ++k)
        if (base + k < count) acc += ld(base + k);
    uint32_t tot;
    block_exclusive<SCAN_THREADS>(acc, s_tmp, &tot);
    if (threadIdx.x == 0) block_sums[blockIdx.x] = tot;
}

// Single-block exclusive scan of the block sums, total to *total (int64):
// each of the TOP_THREADS threads takes a contiguous run of sums.
__global__ void __launch_bounds__(TOP_THREADS) k_scan_top(uint32_t* block_sums, int nblocks, int64_t* total) {
    __shared__ uint32_t s_tmp[TOP_THREADS / kWave];
    const int per = (nblocks + TOP_THREADS - 1) / TOP_THREADS;
    const int b0 = min(nblocks, (int)threadIdx.x * per), b1 = min(nblocks, b0 + per);
    uint32_t sum = 0;
    for (int b = b0; b < b1; ++b) sum += block_sums[b];
    uint32_t tot;
    uint32_t run = block_exclusive<TOP_THREADS>(sum, s_tmp, &tot);
    for (int b = b0; b < b1; ++b) {
        const uint32_t v = block_sums[b];
        block_sums[b] = run;
        run += v;
    }
    if (threadIdx.x == 0 && total != nullptr) *total = (int64_t)tot;
}

template <class Load>
__global__ void __launch_bounds__(SCAN_THREADS) k_scan_final(Load ld, const int64_t* count_dev, int64_t n_max,
                                                             const uint32_t* block_sums, uint32_t* out) {
    __shared__ uint32_t s_tmp[SCAN_THREADS / kWave];
    const int64_t count = eff_count(count_dev, n_max);
    const int64_t base = (int64_t)blockIdx.x * SCAN_TILE + (int64_t)threadIdx.x * SCAN_ITEMS;
    if ((int64_t)blockIdx.x * SCAN_TILE >= count) return;  // whole block beyond the count
    uint32_t v[SCAN_ITEMS];
    uint32_t acc = 0;
#pragma unroll
    for (int k = 0; k < SCAN_ITEMS; ++k) {
        v[k] = (base + k < count) ? ld(base + k) : 0u;
        acc += v[k];
    }
    uint32_t tot;
    uint32_t run = block_sums[blockIdx.x] + block_exclusive<SCAN_THREADS>(acc, s_tmp, &tot);
#pragma unroll
    for (int k = 0; k < SCAN_ITEMS; ++k) {
        if (base + k < count) out[base + k] = run;
        run += v[k];
    }
}

template <class Load>
hipError_t exclusive_scan(Load ld, const int64_t* count_dev, int64_t n_max, uint32_t* block_sums, uint32_t* out,
                          int64_t* total, hipStream_t s) {
    const int nb = (int)((n_max + SCAN_TILE - 1) / SCAN_TILE);
    if (nb == 0) {
        if (total) {
            hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(TOP_THREADS), 0, s, block_sums, 0, total);
        }
        return hipGetLastError();
    }
    hipLaunchKernelGGL(k_scan_partial<Load>, dim3(nb), dim3(SCAN_THREADS), 0, s, ld, count_dev, n_max, block_sums);
    hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(TOP_THREADS), 0, s, block_sums, nb, total);
    hipLaunchKernelGGL(k_scan_final<Load>, dim3(nb), dim3(SCAN_THREADS), 0, s, ld, count_dev, n_max, block_sums,
                       out);
    return hipGetLastError();
}

// ----------------------------------------------------------------------------
// stable LSD radix sort of (u32 key, u32 value), 8-bit digits
// ----------------------------------------------------------------------------
// Lanes of the wave holding the same digit (8 ballots, one per digit bit).
__device__ __forceinline__ uint64_t match_digit(uint32_t d, bool valid) {
    uint64_t m = __ballot(valid);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
        const bool bit = (d >> b) & 1u;
        const uint64_t bb = __ballot(bit);
        m &= bit ? bb : ~bb;
    }
    return m;
}

__global__ void __launch_bounds__(RS_THREADS) k_radix_hist(const uint32_t* __restrict__ keys, const int64_t* count_dev,
                                                           int64_t n_max, int shift, uint32_t* __restrict__ hist,
                                                           int nblk) {
    __shared__ uint32_t h[256];
    const int tid = threadIdx.x, lane = tid & (kWave - 1);
    h[tid] = 0;
    __syncthreads();
    int64_t lo, hi;
    rs_chunk(eff_count(count_dev, n_max), nblk, lo, hi);
    const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    for (int64_t i0 = lo; i0 < hi; i0 += RS_THREADS) {
        const int64_t i = i0 + tid;
        const bool valid = i < hi;
        const uint32_t d = valid ? ((keys[i] >> shift) & 0xffu) : 0u;
        const uint64_t peers = match_digit(d, valid);
        if (valid && (peers & lt) == 0) atomicAdd(&h[d], (uint32_t)__popcll(peers));
    }
    __syncthreads();
    hist[(int64_t)tid * nblk + blockIdx.x] = h[tid];
}

__global__ void __launch_bounds__(RS_THREADS) k_radix_scatter(const uint32_t* __restrict__ keys_in,
                                                              const uint32_t* __restrict__ vals_in,
                                                              const int64_t* count_dev, int64_t n_max, int shift,
                                                              const uint32_t* __restrict__ offs, int nblk,
                                                              uint32_t* __restrict__ keys_out,
                                                              uint32_t* __restrict__ vals_out) {
    __shared__ uint32_t s_base[256];
    __shared__ uint32_t s_wcnt[RS_WAVES][256];
    const int tid = threadIdx.x, lane = tid & (kWave - 1), wave = tid / kWave;
    int64_t lo, hi;
    rs_chunk(eff_count(count_dev, n_max), nblk, lo, hi);
    if (lo >= hi) return;  // uniform across the block
    s_base[tid] = offs[(int64_t)tid * nblk + blockIdx.x];
#pragma unroll
    for (int w = 0; w < RS_WAVES; ++w) s_wcnt[w][tid] = 0;
    __syncthreads();
    const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    for (int64_t i0 = lo; i0 < hi; i0 += RS_THREADS) {
        const int64_t i = i0 + tid;
        const bool valid = i < hi;
        const uint32_t key = valid ? keys_in[i] : 0u;
        const uint32_t val = valid ? vals_in[i] : 0u;
        const uint32_t d = (key >> shift) & 0xffu;
        const uint64_t peers = match_digit(d, valid);
        const uint32_t rank = (uint32_t)__popcll(peers & lt);
        if (valid && rank == 0) s_wcnt[wave][d] = (uint32_t)__popcll(peers);
        __syncthreads();
        if (valid) {
            uint32_t off = s_base[d] + rank;
            for (int w = 0; w < wave; ++w) off += s_wcnt[w][d];
            keys_out[off] = key;
            vals_out[off] = val;
        }
        __syncthreads();
        uint32_t add = 0;
#pragma unroll
        for (int w = 0; w < RS_WAVES; ++w) {
            add += s_wcnt[w][tid];
            s_wcnt[w][tid] = 0;
        }
        s_base[tid] += add;
        __syncthreads();
    }
}

// Sorts (keys, vals) in place over `passes` 8-bit digits starting at bit 0,
// ping-ponging with (keys2, vals2); an even pass count ends in (keys, vals).
hipError_t radix_sort(uint32_t* keys, uint32_t* vals, uint32_t* keys2, uint32_t* vals2, const int64_t* count_dev,
                      int64_t n_max, int passes, uint32_t* hist, uint32_t* block_sums, hipStream_t s) {
    if (n_max <= 0) return hipSuccess;
    const int nblk = rs_blocks(n_max);
    uint32_t *ki = keys, *vi = vals, *ko = keys2, *vo = vals2;
    for (int p = 0; p < passes; ++p) {
        const int shift = 8 * p;
        hipLaunchKernelGGL(k_radix_hist, dim3(nblk), dim3(RS_THREADS), 0, s, ki, count_dev, n_max, shift, hist, nblk);
        hipError_t e = exclusive_scan(LoadU32{hist}, nullptr, (int64_t)256 * nblk, block_sums, hist, nullptr, s);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(k_radix_scatter, dim3(nblk), dim3(RS_THREADS), 0, s, ki, vi, count_dev, n_max, shift, hist,
                           nblk, ko, vo);
        uint32_t* t = ki; ki = ko; ko = t;
        t = vi; vi = vo; vo = t;
    }
    return hipGetLastError();
}

// ----------------------------------------------------------------------------
// pipeline kernels
// ----------------------------------------------------------------------------
// Order-preserving compaction of the visible pairs in three steps: the
// visible count of each run of CV_RUN consecutive pairs, an exclusive scan
// of those counts (one block), then each run ranks its pairs with ballots
// and writes (depth bits, pair index) at its offset.
constexpr int CV_THREADS = 256;
constexpr int CV_RUN = 1024;

__global__ void __launch_bounds__(CV_THREADS) k_count_visible(const int32_t* __restrict__ touched, int64_t vn,
                                                              uint32_t* __restrict__ run_counts) {
    __shared__ uint32_t s_w[CV_THREADS / kWave];
    const int tid = threadIdx.x, lane = tid & (kWave - 1), wave = tid / kWave;
    const int64_t base = (int64_t)blockIdx.x * CV_RUN;
    uint32_t c = 0;
#pragma unroll
    for (int k = 0; k < CV_RUN / CV_THREADS; ++k) {
        const int64_t i = base + k * CV_THREADS + tid;
        c += (i < vn && touched[i] > 0) ? 1u : 0u;
    }
    for (int d = kWave / 2; d > 0; d >>= 1) c += __shfl_xor(c, d, kWave);
    if (lane == 0) s_w[wave] = c;
    __syncthreads();
    if (tid == 0) {
        uint32_t t = 0;
        for (int w = 0; w < CV_THREADS / kWave; ++w) t += s_w[w];
        run_counts[blockIdx.x] = t;
    }
}

__global__ void __launch_bounds__(CV_THREADS) k_compact_visible(const int32_t* __restrict__ touched,
                                                                const float4* __restrict__ rec,
                                                                const uint32_t* __restrict__ run_offs, int64_t vn,
                                                                uint32_t* __restrict__ keys,
                                                                uint32_t* __restrict__ vals) {
    __shared__ uint32_t s_w[CV_THREADS / kWave];
    const int tid = threadIdx.x, lane = tid & (kWave - 1), wave = tid / kWave;
    const int64_t base = (int64_t)blockIdx.x * CV_RUN;
    const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    uint32_t run = run_offs[blockIdx.x];
#pragma unroll
    for (int k = 0; k < CV_RUN / CV_THREADS; ++k) {
        const int64_t i = base + k * CV_THREADS + tid;
        const bool vis = i < vn && touched[i] > 0;
        const uint64_t m = __ballot(vis);
        if (lane == 0) s_w[wave] = (uint32_t)__popcll(m);
        __syncthreads();
        uint32_t off = run, tot = 0;
#pragma unroll
        for (int w = 0; w < CV_THREADS / kWave; ++w) {
            if (w < wave) off += s_w[w];
            tot += s_w[w];
        }
        if (vis) {
            const uint32_t p = off + (uint32_t)__popcll(m & lt);
            keys[p] = __float_as_uint(rec[2 * i + 1].z);  // camera depth, positive: bits are monotone
            vals[p] = (uint32_t)i;
        }
        run += tot;
        __syncthreads();
    }
}

__global__ void k_counts(const int64_t* n_inst, const int64_t* n_vis, int64_t capacity, int64_t* counts,
                         int64_t* n_clamped) {
    if (threadIdx.x != 0) return;
    const int64_t I = *n_inst;
    counts[0] = I;
    counts[1] = *n_vis;
    counts[2] = I > capacity ? 1 : 0;
    counts[3] = 0;
    *n_clamped = I < capacity ? I : capacity;
}

// Emission: the visible pair at depth-sorted position i writes one instance
// per tile of its rectangle at emission indices offs[i] .. offs[i] + touched - 1
// (row-major over the rectangle): key = global tile id, value = the emission
// index itself.  inst_gid[e] keeps the Gaussian of emission index e,
// pair_first[pair] the first emission index of the pair, so that the
// instances of one (view, Gaussian) pair stay contiguous in emission space
// after the tile sort has reordered them.
// Each wavefront takes 64 consecutive pairs and its lanes stride over all of
// their instances together (the pair of instance k found by binary search
// over the pairs' starts in LDS), so a pair with many tiles does not stall
// its wavefront and the writes are contiguous across lanes.
__global__ void __launch_bounds__(256) k_emit(const uint32_t* __restrict__ vis_vals,
                                              const uint32_t* __restrict__ offs, const int64_t* n_vis,
                                              const uint2* __restrict__ rect, const gs_view* __restrict__ views,
                                              int n, int tile, int64_t capacity, uint32_t* __restrict__ keys,
                                              uint32_t* __restrict__ vals, int32_t* __restrict__ inst_gid,
                                              int32_t* __restrict__ pair_first) {
    __shared__ uint32_t s_start[4][kWave];
    __shared__ uint4 s_info[4][kWave];  // (x0 | y0 << 16, rect width, tile base, tiles per row)
    __shared__ int32_t s_gid[4][kWave];
    const int tid = threadIdx.x, lane = tid & (kWave - 1), wave = tid / kWave;
    const int64_t nv = *n_vis;
    const int64_t i0 = (int64_t)blockIdx.x * blockDim.x + (int64_t)wave * kWave;
    if (i0 >= nv) return;  // uniform across the wavefront
    const int64_t i = i0 + lane;
    const bool valid = i < nv;
    int64_t o_i = 0, end_i = 0;
    if (valid) {
        const uint32_t pair = vis_vals[i];
        const int v = (int)(pair / (uint32_t)n);
        const uint32_t gid = pair - (uint32_t)v * (uint32_t)n;
        const uint2 r = rect[pair];
        const uint32_t x0 = r.x & 0xffffu, y0 = r.x >> 16, x1 = r.y & 0xffffu, y1 = r.y >> 16;
        const uint32_t wr = x1 - x0 + 1, hr = y1 - y0 + 1;
        o_i = offs[i];
        end_i = o_i + (int64_t)wr * hr;
        pair_first[pair] = (int32_t)o_i;
        s_info[wave][lane] = make_uint4(x0 | (y0 << 16), wr, (uint32_t)views[v].tile_offset,
                                        (uint32_t)ceil_div(views[v].width, tile));
        s_gid[wave][lane] = (int32_t)gid;
    }
    const int64_t o_w = __shfl(o_i, 0, kWave);  // lane 0 is valid
    s_start[wave][lane] = (uint32_t)(o_i - o_w);
    const int nvalid = (int)__popcll(__ballot(valid));
    const int64_t total = __shfl(end_i, nvalid - 1, kWave) - o_w;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    for (int64_t k = lane; k < total; k += kWave) {
        int lo = 0, hi = nvalid - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if ((int64_t)s_start[wave][mid] <= k) lo = mid;
            else hi = mid - 1;
        }
        const uint4 info = s_info[wave][lo];
        const uint32_t li = (uint32_t)(k - s_start[wave][lo]);
        const uint32_t yy = (info.x >> 16) + li / info.y, xx = (info.x & 0xffffu) + li % info.y;
        const int64_t o = o_w + k;
        if (o < capacity) {
            keys[o] = info.z + yy * info.w + xx;
            vals[o] = (uint32_t)o;
            inst_gid[o] = s_gid[wave][lo];
        }
    }
}

__global__ void k_ranges(const uint32_t* __restrict__ keys, const int64_t* n_inst, int2* __restrict__ ranges) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t I = *n_inst;
    if (i >= I) return;
    const uint32_t k = keys[i];
    if (i == 0 || keys[i - 1] != k) ranges[k].x = (int)i;
    if (i == I - 1 || keys[i + 1] != k) ranges[k].y = (int)(i + 1);
}

struct WsLayout {
    size_t vis_k0, vis_v0, vis_k1, vis_v1, pos, inst_k2, inst_v2, hist, bsum, cnt, total;
};

WsLayout ws_layout(int n, int n_views, int64_t capacity) {
    auto al = [](size_t x) { return (x + 255) & ~(size_t)255; };
    const int64_t vn = (int64_t)n * n_views;
    const int64_t cap = capacity > 0 ? capacity : 1;
    const int64_t big = vn > cap ? vn : cap;
    const int64_t nblk = rs_blocks(big);
    const int64_t scan_n = (256 * nblk > big ? 256 * nblk : big);
    const int64_t nbs = (scan_n + SCAN_TILE - 1) / SCAN_TILE + 1;
    WsLayout L;
    size_t o = 0;
    L.vis_k0 = o; o += al(4 * (size_t)(vn > 0 ? vn : 1));
    L.vis_v0 = o; o += al(4 * (size_t)(vn > 0 ? vn : 1));
    L.vis_k1 = o; o += al(4 * (size_t)(vn > 0 ? vn : 1));
    L.vis_v1 = o; o += al(4 * (size_t)(vn > 0 ? vn : 1));
    L.pos = o; o += al(4 * (size_t)(vn > 0 ? vn : 1));
    L.inst_k2 = o; o += al(4 * (size_t)cap);
    L.inst_v2 = o; o += al(4 * (size_t)cap);
    L.hist = o; o += al(4 * (size_t)(256 * nblk + 1));
    L.bsum = o; o += al(4 * (size_t)nbs);
    L.cnt = o; o += al(8 * 4);
    L.total = o;
    return L;
}

}  // namespace

size_t binsort_workspace_bytes(int n, int n_views, int64_t capacity) { return ws_layout(n, n_views, capacity).total; }

hipError_t launch_binsort(const uint32_t* rect, const int32_t* touched, const float* rec, int n,
                          const gs_view* views_dev, int n_views, int total_tiles, int tile, void* ws,
                          int64_t capacity, uint32_t* tile_keys, int32_t* inst, int32_t* inst_gid,
                          int32_t* pair_first, int32_t* ranges, int64_t* counts, hipStream_t s) {
    const WsLayout L = ws_layout(n, n_views, capacity);
    char* w = static_cast<char*>(ws);
    uint32_t* vis_k0 = reinterpret_cast<uint32_t*>(w + L.vis_k0);
    uint32_t* vis_v0 = reinterpret_cast<uint32_t*>(w + L.vis_v0);
    uint32_t* vis_k1 = reinterpret_cast<uint32_t*>(w + L.vis_k1);
    uint32_t* vis_v1 = reinterpret_cast<uint32_t*>(w + L.vis_v1);
    uint32_t* pos = reinterpret_cast<uint32_t*>(w + L.pos);
    uint32_t* ik2 = reinterpret_cast<uint32_t*>(w + L.inst_k2);
    uint32_t* iv2 = reinterpret_cast<uint32_t*>(w + L.inst_v2);
    uint32_t* hist = reinterpret_cast<uint32_t*>(w + L.hist);
    uint32_t* bsum = reinterpret_cast<uint32_t*>(w + L.bsum);
    int64_t* cnt = reinterpret_cast<int64_t*>(w + L.cnt);  // [0] n_vis [1] n_inst [2] clamped
    const int64_t vn = (int64_t)n * n_views;
    hipError_t e;

    // 1. order-preserving compaction of the visible pairs, key = depth bits
    if (vn > 0) {
        const unsigned nrun = (unsigned)((vn + CV_RUN - 1) / CV_RUN);
        hipLaunchKernelGGL(k_count_visible, dim3(nrun), dim3(CV_THREADS), 0, s, touched, vn, pos);
        hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(TOP_THREADS), 0, s, pos, (int)nrun, &cnt[0]);
        hipLaunchKernelGGL(k_compact_visible, dim3(nrun), dim3(CV_THREADS), 0, s, touched,
                           reinterpret_cast<const float4*>(rec), pos, vn, vis_k0, vis_v0);
    } else {
        hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(TOP_THREADS), 0, s, pos, 0, &cnt[0]);
    }
    // 2. stable sort of the visible pairs by depth (32 bits)
    e = radix_sort(vis_k0, vis_v0, vis_k1, vis_v1, &cnt[0], vn, 4, hist, bsum, s);
    if (e != hipSuccess) return e;
    // 3. instance offsets in depth order, total instance count
    e = exclusive_scan(LoadGatherTouched{touched, vis_v0}, &cnt[0], vn, bsum, pos, &cnt[1], s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_counts, dim3(1), dim3(64), 0, s, &cnt[1], &cnt[0], capacity, counts, &cnt[2]);
    // 4. emission, then stable sort by global tile id
    int bits = 1;
    while ((1ll << bits) < (int64_t)total_tiles) ++bits;
    const int passes = (bits + 7) / 8;
    uint32_t* ek = (passes % 2 == 0) ? reinterpret_cast<uint32_t*>(tile_keys) : ik2;
    uint32_t* ev = (passes % 2 == 0) ? reinterpret_cast<uint32_t*>(inst) : iv2;
    uint32_t* ok = (passes % 2 == 0) ? ik2 : reinterpret_cast<uint32_t*>(tile_keys);
    uint32_t* ov = (passes % 2 == 0) ? iv2 : reinterpret_cast<uint32_t*>(inst);
    if (vn > 0) {
        hipLaunchKernelGGL(k_emit, dim3((unsigned)((vn + 255) / 256)), dim3(256), 0, s, vis_v0, pos, &cnt[0],
                           reinterpret_cast<const uint2*>(rect), views_dev, n, tile, capacity, ek, ev, inst_gid,
                           pair_first);
    }
    e = radix_sort(ek, ev, ok, ov, &cnt[2], capacity, passes, hist, bsum, s);
    if (e != hipSuccess) return e;
    // 5. per-tile [start, end)
    e = fill_u32(reinterpret_cast<uint32_t*>(ranges), 0u, 2 * (int64_t)total_tiles, s);
    if (e != hipSuccess) return e;
    if (capacity > 0) {
        hipLaunchKernelGGL(k_ranges, dim3((unsigned)((capacity + 255) / 256)), dim3(256), 0, s,
                           reinterpret_cast<const uint32_t*>(tile_keys), &cnt[2], reinterpret_cast<int2*>(ranges));
    }
    return hipGetLastError();
}

}  // namespace sgs
