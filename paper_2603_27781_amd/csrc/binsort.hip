// Tile binning and depth sort (GS^3LAM Sec. 3.2.1: the tile-based rasterizer
// of the cited 3DGS work sorts Gaussians in depth order per tile).
//
// Two stable sorts replace one wide-key sort:
//   1. the visible (view, Gaussian) pairs, compacted in (view, index) order,
//      each emit one instance per tile of their rectangle, keyed by global
//      tile id, and the instances are radix-sorted by tile id (ceil(log2
//      tiles) bits; stable, so each tile's list stays in index order);
//   2. each tile's list is sorted by the binary32 bits of its pairs' camera
//      depth, one workgroup per tile (stable counting passes in LDS).
// So the final order is (view, tile, depth bits, Gaussian index).
//
// Every count that the host does not know (visible pairs, instances) stays on
// the device; grids are sized for the capacity and blocks beyond the count
// exit early, so the whole pipeline is graph-capturable.
//
// Prefix sums take one launch where the input is short and two or three
// where it is long.  The radix digit offsets (256 per block) are a single-pass scan with
// decoupled look-back: a block takes a ticket, scans its tile, publishes its
// total and reads the totals of the tiles before it until it meets a
// published prefix; it only ever waits for blocks that took an earlier
// ticket, which are already running, so every wait ends (the spin is bounded
// all the same).  The long scan of the instance offsets (thousands of
// tiles, where such a chain of waits costs more than it saves) writes tile
// totals first, and each tile then sums the totals before it itself; the
// compaction counts runs, scans the run counts in one block and ranks
// inside a run with ballots.
#include <cstdlib>

#include "sgs_common.h"

namespace sgs {

namespace {

// Value of v held by lane (lane ^ J), for wavefront sums and the
// compare-exchanges of the bitonic network.  No LDS round trip where the hardware has a register
// path: J = 1, 2 are DPP quad permutations, J = 8 a DPP row rotation (within
// a row of 16 lanes that is lane ^ 8), J = 16, 32 permlane swaps of v with
// itself (which give the values of the lanes with the bit clear and set);
// J = 4 goes through the LDS crossbar (ds_swizzle, no address operand).
template <int J>
__device__ __forceinline__ uint32_t lane_xor_u32(uint32_t v, int lane) {
    if constexpr (J == 1) {
        return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0xB1, 0xF, 0xF, true);  // quad_perm [1,0,3,2]
    } else if constexpr (J == 2) {
        return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x4E, 0xF, 0xF, true);  // quad_perm [2,3,0,1]
    } else if constexpr (J == 8) {
        return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x128, 0xF, 0xF, true);  // row_ror:8
    } else if constexpr (J == 4) {
        return (uint32_t)__builtin_amdgcn_ds_swizzle((int)v, (4 << 10) | 0x1F);  // xor_mask 4
    } else if constexpr (J == 16) {
        const auto r = __builtin_amdgcn_permlane16_swap(v, v, false, false);  // v(l & ~16), v(l | 16)
        return (lane & 16) ? r[0] : r[1];
    } else {
        static_assert(J == 32, "lane_xor_u32: J is a power of two up to 32");
        const auto r = __builtin_amdgcn_permlane32_swap(v, v, false, false);  // v(l & ~32), v(l | 32)
        return (lane & 32) ? r[0] : r[1];
    }
}

// Value of v in lane l (l wavefront-uniform), read into scalar registers.
__device__ __forceinline__ int64_t read_lane_i64(int64_t v, int l) {
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, l);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)((uint64_t)v >> 32), l);
    return (int64_t)(((uint64_t)hi << 32) | lo);
}

// Sum of x over the 64 lanes, in every lane (integer: the order does not
// matter), with one LDS crossbar step (J = 4) instead of six shuffles.
__device__ __forceinline__ uint32_t wave_sum_u32(uint32_t x, int lane) {
    x += lane_xor_u32<1>(x, lane);
    x += lane_xor_u32<2>(x, lane);
    x += lane_xor_u32<4>(x, lane);
    x += lane_xor_u32<8>(x, lane);
    x += lane_xor_u32<16>(x, lane);
    x += lane_xor_u32<32>(x, lane);
    return x;
}

// Radix passes run on a fixed grid of at most RS_MAXBLK blocks; the device
// side count is split into contiguous chunks (multiples of RS_THREADS), one
// per block, so the digit histograms stay small whatever the capacity and
// only blocks with elements do work.
constexpr int RS_THREADS = 256;
constexpr int RS_MAXBLK = 1024;
constexpr int RS_WAVES = RS_THREADS / kWave;
constexpr int RS_ITEMS = 4;                        // keys per thread per scatter tile
constexpr int RS_TILE = RS_THREADS * RS_ITEMS;     // chunks are whole tiles

int rs_blocks(int64_t n_max) {
    const int64_t b = (n_max + RS_THREADS - 1) / RS_THREADS;
    return (int)(b < RS_MAXBLK ? (b > 0 ? b : 1) : RS_MAXBLK);
}

__device__ __forceinline__ void rs_chunk(int64_t count, int nblk, int64_t& lo, int64_t& hi) {
    const int64_t per = ((count + nblk - 1) / nblk + RS_TILE - 1) / RS_TILE * RS_TILE;
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
struct LoadU32 {
    const uint32_t* p;
    __device__ uint32_t operator()(int64_t i) const { return p[i]; }
};

// Sum of a[0 .. m) by the whole block (all threads get it): used by a block
// to find its offset from the totals of the tiles before it, so that the
// large scans need no top-level scan launch and no waiting between blocks.
// The totals are few (one per tile) and were just written, so they are
// read from L2.
template <int NT>
__device__ __forceinline__ uint32_t block_sum_before(const uint32_t* __restrict__ a, int m, uint32_t* s_tmp) {
    const int tid = threadIdx.x, lane = tid & (kWave - 1), wave = tid / kWave;
    uint32_t x = 0;
    for (int i = tid; i < m; i += NT) x += a[i];
    x = wave_sum_u32(x, lane);
    if (lane == 0) s_tmp[wave] = x;
    __syncthreads();
    uint32_t t = 0;
#pragma unroll
    for (int w = 0; w < NT / kWave; ++w) t += s_tmp[w];
    __syncthreads();
    return t;
}

constexpr int TOP_THREADS = 1024;

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

// Single-pass exclusive scan with decoupled look-back.  Status word of a
// tile: bits 62-63 the state (0 not ready, 1 tile total, 2 inclusive prefix),
// bits 0-31 the value.
constexpr int LB_THREADS = 256;
constexpr int LB_ITEMS = 8;
constexpr int LB_TILE = LB_THREADS * LB_ITEMS;
constexpr uint64_t LB_AGG = 1ull << 62;
constexpr uint64_t LB_INC = 2ull << 62;
constexpr int LB_SPIN_MAX = 1 << 20;

int64_t lb_tiles(int64_t n) { return (n + LB_TILE - 1) / LB_TILE; }

__device__ __forceinline__ void lb_publish(uint64_t* st, uint64_t state, uint32_t value) {
    __hip_atomic_store(st, state | value, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ uint64_t lb_read(const uint64_t* st) {
    return __hip_atomic_load(st, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Where a look-back that gave up is recorded: the call's flag and the
// caller's sticky flag (the low words of counts[3] and counts[4]), and how
// many reads a wait may take.
struct LbGiveUp {
    uint32_t* flag;
    uint32_t* sticky;
    int spin_limit;
};

// Exclusive prefix of tile `tile` (> 0) from the status words of the tiles
// before it; called by one whole wavefront, which reads 64 of them at a
// time, newest first.  Positions before tile 0 count as an inclusive 0.
// A predecessor that has not published after gu.spin_limit further reads is
// counted as 0 -- a short prefix -- and the give-up is recorded, so that the
// binning's later kernels stand down and the caller sees it.
__device__ uint32_t lb_lookback(const uint64_t* status, int tile, LbGiveUp gu) {
    const int lane = threadIdx.x & (kWave - 1);
    uint32_t prefix = 0;
    for (int j = tile - 1;; j -= kWave) {
        const int k = j - lane;
        uint64_t s = k >= 0 ? lb_read(status + k) : LB_INC;
        for (int spin = 0; __any((s >> 62) == 0) && spin < gu.spin_limit; ++spin)
            if ((s >> 62) == 0) s = lb_read(status + k);
        if (__any((s >> 62) == 0) && lane == 0) {
            atomicOr(gu.flag, 1u);
            atomicOr(gu.sticky, 1u);
        }
        const uint64_t inc = __ballot((s >> 62) == 2);
        uint32_t v = (uint32_t)s;
        if (inc != 0 && lane > __builtin_ctzll(inc)) v = 0;  // stop at the nearest inclusive prefix
        v = wave_sum_u32(v, lane);
        prefix += v;
        if (inc != 0) return prefix;
    }
}

// Ticket, tile scan and look-back shared by the single-pass kernels: returns
// the exclusive prefix of this thread's items (excl added to the tile's
// prefix) and the tile's total; all threads of the block call it.
__device__ __forceinline__ uint32_t lb_block(uint32_t acc, int tile, uint64_t* status, uint32_t* s_tmp,
                                             uint32_t* s_prefix, uint32_t* tile_total, LbGiveUp gu) {
    uint32_t tot;
    const uint32_t excl = block_exclusive<LB_THREADS>(acc, s_tmp, &tot);
    if (threadIdx.x < kWave) {
        const int lane = threadIdx.x;
        uint32_t prefix = 0;
        if (tile == 0) {
            if (lane == 0) lb_publish(status, LB_INC, tot);
        } else {
            if (lane == 0) lb_publish(status + tile, LB_AGG, tot);
            prefix = lb_lookback(status, tile, gu);
            if (lane == 0) lb_publish(status + tile, LB_INC, prefix + tot);
        }
        if (lane == 0) *s_prefix = prefix;
    }
    __syncthreads();
    *tile_total = tot;
    return *s_prefix + excl;
}

__device__ __forceinline__ int lb_ticket(uint32_t* ticket, int* s_tile) {
    if (threadIdx.x == 0) *s_tile = (int)atomicAdd(ticket, 1u);
    __syncthreads();
    return *s_tile;
}

// Instance bookkeeping written by the last tile of the instance-offset scan.
struct CountsOut {
    int64_t* counts;         // (instances, visible pairs, overflow, look-back gave up, sticky)
    int64_t* n_clamped;      // min(instances, capacity)
    const int64_t* n_vis;
    int64_t capacity;
};

// Two-step exclusive scan for long inputs: tile totals, then every tile
// sums the totals before it and scans its own items (no top-level launch,
// no waiting between blocks).  Tiles of LB_TILE items, LB_ITEMS consecutive
// items per thread.
template <class Load>
__global__ void __launch_bounds__(LB_THREADS) k_tile_sums(Load ld, const int64_t* count_dev, int64_t n_max,
                                                          uint32_t* __restrict__ sums) {
    __shared__ uint32_t s_tmp[LB_THREADS / kWave];
    const int64_t count = eff_count(count_dev, n_max);
    const int64_t tbase = (int64_t)blockIdx.x * LB_TILE;
    if (tbase >= count) return;  // uniform; no later tile reads this sum
    const int64_t base = tbase + (int64_t)threadIdx.x * LB_ITEMS;
    uint32_t acc = 0;
#pragma unroll
    for (int k = 0; k < LB_ITEMS; ++k)
        if (base + k < count) acc += ld(base + k);
    uint32_t tot;
    block_exclusive<LB_THREADS>(acc, s_tmp, &tot);
    if (threadIdx.x == 0) sums[blockIdx.x] = tot;
}

template <class Load>
__global__ void __launch_bounds__(LB_THREADS) k_tile_scan(Load ld, const int64_t* count_dev, int64_t n_max,
                                                          const uint32_t* __restrict__ sums, uint32_t* out,
                                                          int64_t* total, CountsOut co) {
    __shared__ uint32_t s_tmp[LB_THREADS / kWave];
    const int64_t count = eff_count(count_dev, n_max);
    const int64_t tbase = (int64_t)blockIdx.x * LB_TILE;
    if (tbase >= count && blockIdx.x != 0) return;  // uniform
    const uint32_t prefix = block_sum_before<LB_THREADS>(sums, (int)blockIdx.x, s_tmp);
    const int64_t base = tbase + (int64_t)threadIdx.x * LB_ITEMS;
    uint32_t v[LB_ITEMS];
    uint32_t acc = 0;
#pragma unroll
    for (int k = 0; k < LB_ITEMS; ++k) {
        v[k] = (base + k < count) ? ld(base + k) : 0u;
        acc += v[k];
    }
    uint32_t tot;
    uint32_t run = prefix + block_exclusive<LB_THREADS>(acc, s_tmp, &tot);
#pragma unroll
    for (int k = 0; k < LB_ITEMS; ++k) {
        if (base + k < count) out[base + k] = run;
        run += v[k];
    }
    if (threadIdx.x == 0 && tbase + LB_TILE >= count) {  // the last tile with items (tile 0 if none)
        const int64_t I = (int64_t)prefix + tot;
        if (total != nullptr) *total = I;
        if (co.counts != nullptr) {
            co.counts[0] = I;
            co.counts[1] = *co.n_vis;
            co.counts[2] = I > co.capacity ? 1 : 0;
            co.counts[3] = 0;
            if (I > co.capacity) co.counts[4] |= 1;  // sticky: only the caller clears it
            *co.n_clamped = I < co.capacity ? I : co.capacity;
        }
    }
}

// Exclusive scan of ld(0 .. count) into out (in place allowed: a tile is
// read before it is written and by no other block); *total <- the sum.
// Grid: lb_tiles(n_max) blocks.
template <class Load>
__global__ void __launch_bounds__(LB_THREADS) k_scan_lb(Load ld, const int64_t* count_dev, int64_t n_max,
                                                        uint64_t* status, uint32_t* ticket, uint32_t* out,
                                                        int64_t* total, LbGiveUp gu) {
    __shared__ uint32_t s_tmp[LB_THREADS / kWave];
    __shared__ uint32_t s_prefix;
    __shared__ int s_tile;
    const int tile = lb_ticket(ticket, &s_tile);
    const int64_t count = eff_count(count_dev, n_max);
    const int64_t tbase = (int64_t)tile * LB_TILE;
    if (tbase >= count && tile != 0) return;  // uniform: no later tile reads this one
    const int64_t base = tbase + (int64_t)threadIdx.x * LB_ITEMS;
    uint32_t v[LB_ITEMS];
    uint32_t acc = 0;
#pragma unroll
    for (int k = 0; k < LB_ITEMS; ++k) {
        v[k] = (base + k < count) ? ld(base + k) : 0u;
        acc += v[k];
    }
    uint32_t tot;
    uint32_t run = lb_block(acc, tile, status, s_tmp, &s_prefix, &tot, gu);
#pragma unroll
    for (int k = 0; k < LB_ITEMS; ++k) {
        if (base + k < count) out[base + k] = run;
        run += v[k];
    }
    if (threadIdx.x == 0 && total != nullptr && tbase + LB_TILE >= count) *total = (int64_t)s_prefix + tot;
}

// Single-pass scan for short inputs (few tiles: the look-back stays short).
template <class Load>
hipError_t exclusive_scan(Load ld, const int64_t* count_dev, int64_t n_max, uint64_t* status, uint32_t* ticket,
                          uint32_t* out, int64_t* total, LbGiveUp gu, hipStream_t s) {
    const int64_t nt = lb_tiles(n_max);
    hipLaunchKernelGGL(k_scan_lb<Load>, dim3((unsigned)(nt > 0 ? nt : 1)), dim3(LB_THREADS), 0, s, ld, count_dev,
                       n_max, status, ticket, out, total, gu);
    return hipGetLastError();
}

// Two-step scan for long inputs; sums holds lb_tiles(n_max) words.
template <class Load>
hipError_t exclusive_scan_long(Load ld, const int64_t* count_dev, int64_t n_max, uint32_t* sums, uint32_t* out,
                               int64_t* total, hipStream_t s, CountsOut co) {
    const int64_t nt = lb_tiles(n_max) > 0 ? lb_tiles(n_max) : 1;
    hipLaunchKernelGGL(k_tile_sums<Load>, dim3((unsigned)nt), dim3(LB_THREADS), 0, s, ld, count_dev, n_max, sums);
    hipLaunchKernelGGL(k_tile_scan<Load>, dim3((unsigned)nt), dim3(LB_THREADS), 0, s, ld, count_dev, n_max, sums,
                       out, total, co);
    return hipGetLastError();
}

// Zeroes the look-back status words and tickets of one binning call and the
// per-tile ranges (a fill kernel rather than a memset, so that graph replays
// stay correct).
__global__ void k_bin_reset(uint64_t* status, int64_t n_status, uint32_t* tickets, int n_tickets, uint32_t* ranges,
                            int64_t n_ranges) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n_status; i += stride) status[i] = 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n_ranges; i += stride) ranges[i] = 0;
    if (blockIdx.x == 0 && (int)threadIdx.x < n_tickets) tickets[threadIdx.x] = 0;
}

// ----------------------------------------------------------------------------
// stable LSD radix sort of (u32 key, u32 value), 8-bit digits
// ----------------------------------------------------------------------------
// Key source of a radix pass: the (key, value) arrays of the previous pass.
// (A source may also skip elements, key() returning false: the histogram
// and the scatter then leave them out.)
struct SrcKV {
    const uint32_t* keys;
    const uint32_t* vals;
    __device__ bool key(int64_t i, uint32_t& k) const {
        k = keys[i];
        return true;
    }
    __device__ uint32_t val(int64_t i) const { return vals[i]; }
};
// Key source whose value is the key's own position (the first pass of a
// sort that carries the input order along, so nobody has to write it out).
struct SrcKI {
    const uint32_t* keys;
    __device__ bool key(int64_t i, uint32_t& k) const {
        k = keys[i];
        return true;
    }
    __device__ uint32_t val(int64_t i) const { return (uint32_t)i; }
};
template <class Src>
__global__ void __launch_bounds__(RS_THREADS) k_radix_hist(Src src, const int64_t* count_dev, int64_t n_max,
                                                           int shift, uint32_t* __restrict__ hist, int nblk) {
    __shared__ uint32_t h[256];
    const int tid = threadIdx.x, lane = tid & (kWave - 1);
    h[tid] = 0;
    __syncthreads();
    int64_t lo, hi;
    rs_chunk(eff_count(count_dev, n_max), nblk, lo, hi);
    const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    for (int64_t i0 = lo; i0 < hi; i0 += RS_THREADS) {
        const int64_t i = i0 + tid;
        uint32_t key = 0;
        const bool valid = i < hi && src.key(i, key);
        const uint32_t d = valid ? ((key >> shift) & 0xffu) : 0u;
        const uint64_t peers = match_digit(d, valid);
        if (valid && (peers & lt) == 0) atomicAdd(&h[d], (uint32_t)__popcll(peers));
    }
    __syncthreads();
    hist[(int64_t)tid * nblk + blockIdx.x] = h[tid];
}

// Stable scatter of one pass, a tile of RS_TILE keys at a time: every key is
// ranked inside the tile (wavefront ballots per row of RS_THREADS keys, then
// per digit a prefix over the rows and wavefronts, then over the digits),
// the tile is reordered by digit in LDS, and each digit's run of keys is
// written to its global position as consecutive addresses, instead of every
// key going to a different place.
template <class Src>
__global__ void __launch_bounds__(RS_THREADS) k_radix_scatter(Src src, const int64_t* count_dev, int64_t n_max,
                                                              int shift, const uint32_t* __restrict__ offs,
                                                              int nblk, uint32_t* __restrict__ keys_out,
                                                              uint32_t* __restrict__ vals_out,
                                                              const uint32_t* __restrict__ gave_up) {
    constexpr int SLOTS = RS_ITEMS * RS_WAVES;  // (row, wavefront) slots of a tile
    __shared__ uint32_t s_base[256];             // next global position per digit
    __shared__ uint32_t s_lstart[256];           // first tile position per digit
    __shared__ uint32_t s_cnt[SLOTS][256];       // per slot: count, then offset within the digit
    __shared__ uint32_t s_key[RS_TILE];
    __shared__ uint32_t s_val[RS_TILE];
    __shared__ uint32_t s_tmp[RS_WAVES];
    const int tid = threadIdx.x, lane = tid & (kWave - 1), wave = tid / kWave;
    int64_t lo, hi;
    rs_chunk(eff_count(count_dev, n_max), nblk, lo, hi);
    if (lo >= hi) return;  // uniform across the block
    if (*gave_up) return;  // the digit offsets are not to be trusted (uniform)
    s_base[tid] = offs[(int64_t)tid * nblk + blockIdx.x];
    const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    for (int64_t t0 = lo; t0 < hi; t0 += RS_TILE) {
#pragma unroll
        for (int sl = 0; sl < SLOTS; ++sl) s_cnt[sl][tid] = 0;
        __syncthreads();
        uint32_t key[RS_ITEMS], val[RS_ITEMS], rank[RS_ITEMS];
        bool valid[RS_ITEMS];
#pragma unroll
        for (int k = 0; k < RS_ITEMS; ++k) {
            const int64_t i = t0 + k * RS_THREADS + tid;
            key[k] = 0;
            valid[k] = i < hi && src.key(i, key[k]);
            val[k] = valid[k] ? src.val(i) : 0u;
            const uint32_t d = (key[k] >> shift) & 0xffu;
            const uint64_t peers = match_digit(d, valid[k]);
            rank[k] = (uint32_t)__popcll(peers & lt);
            if (valid[k] && rank[k] == 0) s_cnt[k * RS_WAVES + wave][d] = (uint32_t)__popcll(peers);
        }
        __syncthreads();
        // thread d: offsets of digit d's slots, in tile order
        uint32_t run = 0;
#pragma unroll
        for (int sl = 0; sl < SLOTS; ++sl) {
            const uint32_t c = s_cnt[sl][tid];
            s_cnt[sl][tid] = run;
            run += c;
        }
        uint32_t nvalid;
        s_lstart[tid] = block_exclusive<RS_THREADS>(run, s_tmp, &nvalid);
        __syncthreads();
#pragma unroll
        for (int k = 0; k < RS_ITEMS; ++k) {
            if (valid[k]) {
                const uint32_t d = (key[k] >> shift) & 0xffu;
                const uint32_t p = s_lstart[d] + s_cnt[k * RS_WAVES + wave][d] + rank[k];
                s_key[p] = key[k];
                s_val[p] = val[k];
            }
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < RS_ITEMS; ++k) {
            const uint32_t p = (uint32_t)(k * RS_THREADS + tid);
            if (p < nvalid) {
                const uint32_t kk = s_key[p], vv = s_val[p];
                const uint32_t d = (kk >> shift) & 0xffu;
                const uint32_t g = s_base[d] + (p - s_lstart[d]);
                if (g < n_max) {
                    keys_out[g] = kk;
                    vals_out[g] = vv;
                }
            }
        }
        __syncthreads();
        s_base[tid] += run;
    }
}

// One radix pass from src into (ko, vo): digit histograms, their look-back
// scan (status words and ticket zeroed beforehand; *total <- the number of
// keys that took part), then the stable scatter.
template <class Src>
hipError_t radix_pass(Src src, const int64_t* count_dev, int64_t n_max, int shift, uint32_t* hist,
                      uint64_t* status, uint32_t* ticket, int64_t* total, uint32_t* ko, uint32_t* vo, LbGiveUp gu,
                      hipStream_t s) {
    const int nblk = rs_blocks(n_max);
    hipLaunchKernelGGL(k_radix_hist<Src>, dim3(nblk), dim3(RS_THREADS), 0, s, src, count_dev, n_max, shift, hist,
                       nblk);
    hipError_t e = exclusive_scan(LoadU32{hist}, nullptr, (int64_t)256 * nblk, status, ticket, hist, total, gu, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_radix_scatter<Src>, dim3(nblk), dim3(RS_THREADS), 0, s, src, count_dev, n_max, shift, hist,
                       nblk, ko, vo, gu.flag);
    return hipGetLastError();
}

// Sorts keys over `passes` 8-bit digits starting at bit 0, each key carrying
// its input position as its value (vals is not read), ping-ponging with
// (keys2, vals2); an even pass count ends in (keys, vals).
// Pass p scans its digit offsets with status words status + p * spine_tiles
// and ticket tickets[p] (all zeroed beforehand).
hipError_t radix_sort(uint32_t* keys, uint32_t* vals, uint32_t* keys2, uint32_t* vals2, const int64_t* count_dev,
                      int64_t n_max, int passes, uint32_t* hist, uint64_t* status, int64_t spine_tiles,
                      uint32_t* tickets, LbGiveUp gu, hipStream_t s) {
    if (n_max <= 0) return hipSuccess;
    uint32_t *ki = keys, *vi = vals, *ko = keys2, *vo = vals2;
    for (int p = 0; p < passes; ++p) {
        hipError_t e = (p == 0) ? radix_pass(SrcKI{ki}, count_dev, n_max, 0, hist, status, tickets, nullptr, ko,
                                             vo, gu, s)
                                : radix_pass(SrcKV{ki, vi}, count_dev, n_max, 8 * p, hist,
                                             status + p * spine_tiles, tickets + p, nullptr, ko, vo, gu, s);
        if (e != hipSuccess) return e;
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
// and writes (tile count, pair index) at its offset.
constexpr int CV_THREADS = 256;
constexpr int CV_RUN = 2048;

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
    c = wave_sum_u32(c, lane);
    if (lane == 0) s_w[wave] = c;
    __syncthreads();
    if (tid == 0) {
        uint32_t t = 0;
        for (int w = 0; w < CV_THREADS / kWave; ++w) t += s_w[w];
        run_counts[blockIdx.x] = t;
    }
}

__global__ void __launch_bounds__(CV_THREADS) k_compact_visible(const int32_t* __restrict__ touched,
                                                                const uint32_t* __restrict__ run_offs, int64_t vn,
                                                                uint32_t* __restrict__ counts,
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
            counts[p] = (uint32_t)touched[i];
            vals[p] = (uint32_t)i;
        }
        run += tot;
        __syncthreads();
    }
}

// Emission: the visible pair at compacted position i writes one instance
// per tile of its rectangle at emission indices offs[i] .. offs[i] + touched - 1
// (row-major over the rectangle): key = global tile id (the first tile-sort
// pass attaches the emission index as the value).  inst_gid[e] keeps the Gaussian of emission index e,
// depth_e[e] the binary32 bits of its pair's camera depth (the per-tile sort
// key, read there by emission index instead of through inst_gid and the
// pair's projected record: one gather per instance instead of two dependent
// ones; the projection stores the bits in the pair's rectangle entry, so
// this kernel reads them with the rectangle), pair_first[pair] the first
// emission index of the pair, so that the
// instances of one (view, Gaussian) pair stay contiguous in emission space
// after the tile sort has reordered them.
// Each wavefront takes 64 consecutive pairs and its lanes stride over all of
// their instances together, 64 at a time, so a pair with many tiles does
// not stall its wavefront and the writes are contiguous across lanes.  The
// pair of each instance: every pair whose first instance falls in the
// current 64 marks that slot with its lane in LDS, and a max-scan over the
// wavefront (DPP) carries the latest mark to every later slot.
__global__ void __launch_bounds__(256) k_emit(const uint32_t* __restrict__ vis_vals,
                                              const uint32_t* __restrict__ offs, const int64_t* n_vis,
                                              const uint4* __restrict__ rect, const gs_view* __restrict__ views,
                                              int n, int tile, int64_t capacity,
                                              uint32_t* __restrict__ keys, int32_t* __restrict__ inst_gid,
                                              uint32_t* __restrict__ depth_e, int32_t* __restrict__ pair_first) {
    __shared__ uint32_t s_start[4][kWave];
    __shared__ uint4 s_info[4][kWave];  // (x0 | y0 << 16, rect width, tile base, tiles per row)
    __shared__ int32_t s_gid[4][kWave];
    __shared__ uint32_t s_depth[4][kWave];
    __shared__ int32_t s_mark[4][kWave];
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
        const uint4 r = rect[pair];
        const uint32_t x0 = r.x & 0xffffu, y0 = r.x >> 16, x1 = r.y & 0xffffu, y1 = r.y >> 16;
        const uint32_t wr = x1 - x0 + 1, hr = y1 - y0 + 1;
        o_i = offs[i];
        end_i = o_i + (int64_t)wr * hr;
        pair_first[pair] = (int32_t)o_i;
        s_info[wave][lane] = make_uint4(x0 | (y0 << 16), wr, (uint32_t)views[v].tile_offset,
                                        (uint32_t)ceil_div(views[v].width, tile));
        s_gid[wave][lane] = (int32_t)gid;
        s_depth[wave][lane] = r.z;
    }
    const int64_t o_w = read_lane_i64(o_i, 0);  // lane 0 is valid
    s_start[wave][lane] = (uint32_t)(o_i - o_w);
    const int nvalid = (int)__popcll(__ballot(valid));
    const int64_t total = read_lane_i64(end_i, nvalid - 1) - o_w;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    const int64_t my_start = valid ? o_i - o_w : -1;
    int carry = 0;  // the pair of the last instance before the current 64
    for (int64_t base = 0; base < total; base += kWave) {
        const int64_t k = base + lane;
        s_mark[wave][lane] = -1;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        // starts strictly increase (a visible pair has an instance), so a
        // slot is marked at most once
        if (my_start >= base && my_start < base + kWave) s_mark[wave][my_start - base] = lane;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        const int lo = max(wave_max_scan(s_mark[wave][lane]), carry);
        carry = __builtin_amdgcn_readlane(lo, kWave - 1);
        if (k >= total) continue;
        const uint4 info = s_info[wave][lo];
        const uint32_t li = (uint32_t)(k - s_start[wave][lo]);
        // row and column of instance li in the rectangle (width info.y):
        // the quotient is below 2^16, so a float estimate is within one of
        // it and one correction step makes it exact
        int64_t q = (int64_t)((float)li * __builtin_amdgcn_rcpf((float)info.y));
        int64_t r = (int64_t)li - q * (int64_t)info.y;
        if (r < 0) {
            --q;
            r += info.y;
        } else if (r >= (int64_t)info.y) {
            ++q;
            r -= info.y;
        }
        const uint32_t yy = (info.x >> 16) + (uint32_t)q, xx = (info.x & 0xffffu) + (uint32_t)r;
        const int64_t o = o_w + k;
        if (o < capacity) {
            keys[o] = info.z + yy * info.w + xx;
            inst_gid[o] = s_gid[wave][lo];
            depth_e[o] = s_depth[wave][lo];
        }
    }
}

// Per-tile [start, end) of the sorted instances; nothing (every range left
// empty) when a look-back of the sort gave up.
__global__ void k_ranges(const uint32_t* __restrict__ keys, const int64_t* n_inst, int2* __restrict__ ranges,
                         const uint32_t* __restrict__ gave_up) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t I = *n_inst;
    if (i >= I || *gave_up) return;
    const uint32_t k = keys[i];
    if (i == 0 || keys[i - 1] != k) ranges[k].x = (int)i;
    if (i == I - 1 || keys[i + 1] != k) ranges[k].y = (int)(i + 1);
}

// Per-tile depth order.  The visible pairs are emitted in (view, index)
// order and the tile sort is stable, so each tile's instances arrive in
// Gaussian-index order; a stable sort of each tile's list by the binary32
// bits of its pair's camera depth (positive, so the bits order like the
// values) leaves them in (depth, index) order, the order the forward and
// backward walk.  The sort key of the instance at list position i is
// (depth bits << 32 | i): distinct keys, so any correct sort is the stable
// one.  A list is cut into runs of 64 keys, one key per lane; each run is
// sorted across the lanes of a wavefront by a bitonic network; the rank of
// a key among up to eight runs (a chunk of 512) is its lane plus, for every
// other run, the number of that run's keys below it (a 6-step binary search
// in LDS); chunks of a longer list merge the same way (8- or 9-step
// searches in the other sorted chunks).  k_tile_sort_short gives each list of up to
// kTsShort one wavefront; k_tile_sort_long gives each longer list a
// workgroup, in LDS up to kTsLong, and beyond that (rare) stable counting
// passes over 8-bit digits in global memory (the tile's slices of the
// sorted tile keys, whose values are all the tile's own id and are written
// back, and of the tile sort's ping-pong arrays, unused by then).
constexpr int kTsShort = 512, kTsLong = 4096;
constexpr int kTsChunk = 512;  // keys a wavefront sorts at once (8 runs of 64)

template <int NT>
struct SegSortLds {
    uint32_t next[256];             // next output position per digit
    uint32_t wcnt[NT / kWave][256];  // per chunk: each wavefront's count per digit
    uint32_t tmp[NT / kWave];
};

// One stable counting pass of the whole block over the digit at `shift`:
// (kin, vin) -> (kout, vout), L items, every array in LDS or every array in
// global memory.  Chunks of NT items: ranks within a wavefront from ballots,
// wavefronts in order, chunks in order.  Thread tid keeps the digits
// tid * DPT .. tid * DPT + DPT - 1 of the tables.
template <int NT>
__device__ void seg_pass(const uint32_t* kin, const uint32_t* vin, uint32_t* kout, uint32_t* vout, int L, int shift,
                         SegSortLds<NT>& S) {
    constexpr int DPT = 256 / NT, NW = NT / kWave;
    const int tid = threadIdx.x, lane = tid & (kWave - 1), wave = tid / kWave;
#pragma unroll
    for (int q = 0; q < DPT; ++q) S.next[tid * DPT + q] = 0;
    __syncthreads();
    const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    for (int c0 = 0; c0 < L; c0 += NT) {
        // one LDS atomic per run of equal digits in a wavefront (the keys of
        // a tile share most of their high bits)
        const int i = c0 + tid;
        const bool valid = i < L;
        const uint32_t d = valid ? (kin[i] >> shift) & 0xffu : 0u;
        const uint64_t peers = match_digit(d, valid);
        if (valid && (peers & lt) == 0) atomicAdd(&S.next[d], (uint32_t)__popcll(peers));
    }
    __syncthreads();
    uint32_t c[DPT], sum = 0;
#pragma unroll
    for (int q = 0; q < DPT; ++q) {
        c[q] = S.next[tid * DPT + q];
        sum += c[q];
    }
    uint32_t tot;
    uint32_t run = block_exclusive<NT>(sum, S.tmp, &tot);  // barriers inside
#pragma unroll
    for (int q = 0; q < DPT; ++q) {
        S.next[tid * DPT + q] = run;
        run += c[q];
    }
    for (int c0 = 0; c0 < L; c0 += NT) {
#pragma unroll
        for (int w = 0; w < NW; ++w)
#pragma unroll
            for (int q = 0; q < DPT; ++q) S.wcnt[w][tid * DPT + q] = 0;
        __syncthreads();
        const int i = c0 + tid;
        const bool valid = i < L;
        const uint32_t k = valid ? kin[i] : 0u, v = valid ? vin[i] : 0u;
        const uint32_t d = (k >> shift) & 0xffu;
        const uint64_t peers = match_digit(d, valid);
        const uint32_t rank = (uint32_t)__popcll(peers & lt);
        if (valid && rank == 0) S.wcnt[wave][d] = (uint32_t)__popcll(peers);
        __syncthreads();
        if (valid) {
            uint32_t o = S.next[d] + rank;
            for (int w = 0; w < wave; ++w) o += S.wcnt[w][d];
            kout[o] = k;
            vout[o] = v;
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < DPT; ++q) {
            uint32_t add = 0;
#pragma unroll
            for (int w = 0; w < NW; ++w) add += S.wcnt[w][tid * DPT + q];
            S.next[tid * DPT + q] += add;
        }
    }
}

constexpr int TSS_THREADS = kWave;  // short lists: one wavefront per tile
constexpr int TSL_THREADS = 256;    // long lists: one workgroup per tile
constexpr uint64_t kNoKey = ~0ull;  // padding, above every real key

template <int J>
__device__ __forceinline__ uint64_t lane_xor_u64(uint64_t v, int lane) {
    const uint32_t lo = lane_xor_u32<J>((uint32_t)v, lane);
    const uint32_t hi = lane_xor_u32<J>((uint32_t)(v >> 32), lane);
    return ((uint64_t)hi << 32) | lo;
}

// Bitonic sort of one key per lane: afterwards lane l holds the l-th
// smallest of the wavefront's 64 keys.  Blocks of SIZE = 2, 4, ..., 64, each
// merged by compare-exchanges at distances J = SIZE/2, ..., 1; in each, the
// lane with bit J clear keeps the smaller key inside an ascending block (bit
// SIZE clear) and the larger inside a descending one.
template <int SIZE, int J>
__device__ __forceinline__ uint64_t bitonic_merge(uint64_t x, int lane) {
    const uint64_t y = lane_xor_u64<J>(x, lane);
    const bool keep_min = ((lane & J) == 0) == ((lane & SIZE) == 0);
    x = keep_min ? (y < x ? y : x) : (y > x ? y : x);
    if constexpr (J > 1) x = bitonic_merge<SIZE, J / 2>(x, lane);
    return x;
}

template <int SIZE>
__device__ __forceinline__ uint64_t bitonic_sort(uint64_t x, int lane) {
    if constexpr (SIZE > 2) x = bitonic_sort<SIZE / 2>(x, lane);
    return bitonic_merge<SIZE, SIZE / 2>(x, lane);
}

__device__ __forceinline__ uint64_t wave_bitonic_u64(uint64_t x, int lane) { return bitonic_sort<kWave>(x, lane); }

// Number of keys of the sorted array a[0 .. 2^LOG) below `key`
// (branch-free binary search; a is padded with kNoKey).
template <int LOG>
__device__ __forceinline__ int count_below(const uint64_t* a, uint64_t key) {
    int p = 0;
#pragma unroll
    for (int s = 1 << (LOG - 1); s > 0; s >>= 1) p += a[p + s - 1] < key ? s : 0;
    return p + (a[p] < key ? 1 : 0);
}

// One wavefront sorts the keys k[0 .. R) (run r holds list positions
// r*64 .. r*64+63, kNoKey past the end): every run across the lanes, the
// runs stored in s_run, then each key's rank among all R runs.  Returns, in
// k[r], the sorted keys of run r and, in rank[r], their ranks in the chunk.
template <int R>
__device__ __forceinline__ void wave_sort_chunk(uint64_t (&k)[8], int (&rank)[8], uint64_t* s_run, int lane) {
#pragma unroll
    for (int r = 0; r < R; ++r) {
        k[r] = wave_bitonic_u64(k[r], lane);
        s_run[r * kWave + lane] = k[r];
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll
    for (int r = 0; r < R; ++r) {
        int rk = lane;
#pragma unroll
        for (int r2 = 0; r2 < R; ++r2)
            if (r2 != r) rk += count_below<6>(s_run + r2 * kWave, k[r]);
        rank[r] = rk;
    }
}

// Runs R of a chunk of n keys, dispatched to a compile-time count.
__device__ __forceinline__ void wave_sort_chunk_n(int n, uint64_t (&k)[8], int (&rank)[8], uint64_t* s_run,
                                                  int lane) {
    switch ((n + kWave - 1) / kWave) {
        case 1: wave_sort_chunk<1>(k, rank, s_run, lane); break;
        case 2: wave_sort_chunk<2>(k, rank, s_run, lane); break;
        case 3: wave_sort_chunk<3>(k, rank, s_run, lane); break;
        case 4: wave_sort_chunk<4>(k, rank, s_run, lane); break;
        case 5: wave_sort_chunk<5>(k, rank, s_run, lane); break;
        case 6: wave_sort_chunk<6>(k, rank, s_run, lane); break;
        case 7: wave_sort_chunk<7>(k, rank, s_run, lane); break;
        default: wave_sort_chunk<8>(k, rank, s_run, lane); break;
    }
}

// Sort key of list position i of the tile: (depth bits << 32) | i.
__device__ __forceinline__ uint64_t depth_key(const uint32_t* __restrict__ depth_e, uint32_t e, int i) {
    return ((uint64_t)depth_e[e] << 32) | (uint32_t)i;
}

// Tiles in the XCD-aware order of the compositing launches (tile_of_block).
__global__ void __launch_bounds__(TSS_THREADS) k_tile_sort_short(const int2* __restrict__ ranges, int total_tiles,
                                                                  int run, const uint32_t* __restrict__ depth_e,
                                                                  int32_t* __restrict__ inst,
                                                                  uint32_t* __restrict__ long_list,
                                                                  uint32_t* __restrict__ long_count,
                                                                  const uint32_t* __restrict__ gave_up) {
    static_assert(kTsShort == kTsChunk && kTsChunk == 8 * kWave, "a short list is one chunk of eight runs");
    __shared__ uint64_t s_run[kTsChunk];
    __shared__ uint32_t s_e[kTsShort];
    const int t = tile_of_block(blockIdx.x, total_tiles, run);
    if (t < 0 || *gave_up) return;  // after a look-back gave up the lists are not sorted (and none is long)
    const int2 rg = ranges[t];
    const int L = rg.y - rg.x;
    if (L > kTsShort) {  // uniform across the wavefront: left to k_tile_sort_long
        if (threadIdx.x == 0) long_list[atomicAdd(long_count, 1u)] = (uint32_t)t;
        return;
    }
    if (L <= 1) return;
    const int lane = threadIdx.x;
    uint32_t* einst = reinterpret_cast<uint32_t*>(inst) + rg.x;
    uint64_t k[8];
    int rank[8];
#pragma unroll
    for (int r = 0; r < 8; ++r) {
        const int i = r * kWave + lane;
        k[r] = kNoKey;
        if (i < L) {
            const uint32_t e = einst[i];
            s_e[i] = e;
            k[r] = depth_key(depth_e, e, i);
        }
    }
    wave_sort_chunk_n(L, k, rank, s_run, lane);
    // s_e was written by other lanes of this (only) wavefront
    __syncthreads();
#pragma unroll
    for (int r = 0; r < 8; ++r)
        if (r * kWave < L && k[r] != kNoKey) einst[rank[r]] = s_e[(uint32_t)k[r]];
}

// One long list (tile t, more than kTsShort instances), by the whole block.
__device__ void sort_long_list(int t, const int2* __restrict__ ranges, const uint32_t* __restrict__ depth_e,
                               uint32_t* __restrict__ tile_keys,
                               int32_t* __restrict__ inst, uint32_t* __restrict__ gk, uint32_t* __restrict__ gv,
                               uint64_t (&s_sorted)[kTsLong], uint64_t (&s_run)[TSL_THREADS / kWave][kTsChunk],
                               uint32_t (&s_e)[kTsLong], SegSortLds<TSL_THREADS>& S) {
    constexpr int NW = TSL_THREADS / kWave;
    const int2 rg = ranges[t];
    const int L = rg.y - rg.x;
    uint32_t* einst = reinterpret_cast<uint32_t*>(inst) + rg.x;
    const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
    if (L <= kTsLong) {
        // chunks of 256 keys (four runs) up to 1024, so that all four
        // wavefronts sort; of 512 beyond, where more chunks would make the
        // final merge's searches the larger cost
        const bool small = L <= 4 * (kTsChunk / 2);
        const int CH = small ? kTsChunk / 2 : kTsChunk;
        const int nchunk = (L + CH - 1) / CH;
        for (int c = wave; c < nchunk; c += NW) {
            const int c0 = c * CH;
            const int nc = min(CH, L - c0);
            uint64_t k[8];
            int rank[8];
#pragma unroll
            for (int r = 0; r < 8; ++r) {
                const int i = c0 + r * kWave + lane;
                k[r] = kNoKey;
                if (r * kWave < CH && i < L) {
                    const uint32_t e = einst[i];
                    s_e[i] = e;
                    k[r] = depth_key(depth_e, e, i);
                }
            }
            wave_sort_chunk_n(nc, k, rank, s_run[wave], lane);
#pragma unroll
            for (int r = 0; r < 8; ++r)
                if (r * kWave + lane < nc) s_sorted[c0 + rank[r]] = k[r];
            // pad the last chunk to a full CH for the searches
            for (int i = nc + lane; i < CH; i += kWave) s_sorted[c0 + i] = kNoKey;
            // s_run is rewritten by this wavefront's next chunk
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        }
        __syncthreads();
        for (int j = threadIdx.x; j < L; j += TSL_THREADS) {
            const uint64_t key = s_sorted[j];
            const int c = j / CH;
            int pos = j - c * CH;
            for (int c2 = 0; c2 < nchunk; ++c2) {
                if (c2 == c) continue;
                pos += small ? count_below<8>(s_sorted + c2 * CH, key) : count_below<9>(s_sorted + c2 * CH, key);
            }
            einst[pos] = s_e[(uint32_t)key];
        }
        return;
    }
    // in global memory: (depth bits, emission index) start in (tile_keys,
    // inst) and ping-pong with the scratch slices; after four passes they
    // are back
    uint32_t* bk = tile_keys + rg.x;
    uint32_t* ak = gk + rg.x;
    uint32_t* av = gv + rg.x;
    for (int i = threadIdx.x; i < L; i += TSL_THREADS)
        bk[i] = depth_e[einst[i]];
#pragma unroll
    for (int p = 0; p < 4; ++p) {
        // the previous pass's global writes are complete and visible to the
        // whole block (and not stale in this CU's cache) before they are read
        __threadfence();
        __syncthreads();
        if (p & 1) seg_pass<TSL_THREADS>(ak, av, bk, einst, L, 8 * p, S);
        else seg_pass<TSL_THREADS>(bk, einst, ak, av, L, 8 * p, S);
    }
    __threadfence();
    __syncthreads();
    for (int i = threadIdx.x; i < L; i += TSL_THREADS) bk[i] = (uint32_t)t;
}

// The lists longer than kTsShort, which k_tile_sort_short listed in
// long_list: a fixed grid of workgroups walks the list, one tile each at a
// time.  Up to kTsLong: each wavefront sorts chunks (wave_sort_chunk) of 256
// keys for lists up to 1024, else of 512, into s_sorted (the last chunk
// padded with kNoKey), then every key's place
// is its rank in its chunk plus, for each other chunk, the number of that
// chunk's keys below it.  Beyond kTsLong: stable counting passes over the
// four bytes of the depth bits in global memory.
__global__ void __launch_bounds__(TSL_THREADS) k_tile_sort_long(const int2* __restrict__ ranges,
                                                                 const uint32_t* __restrict__ long_list,
                                                                 const uint32_t* __restrict__ long_count,
                                                                 const uint32_t* __restrict__ depth_e,
                                                                 uint32_t* __restrict__ tile_keys,
                                                                 int32_t* __restrict__ inst,
                                                                 uint32_t* __restrict__ gk,
                                                                 uint32_t* __restrict__ gv) {
    __shared__ uint64_t s_sorted[kTsLong];
    __shared__ uint64_t s_run[TSL_THREADS / kWave][kTsChunk];
    __shared__ uint32_t s_e[kTsLong];
    __shared__ SegSortLds<TSL_THREADS> S;
    const uint32_t count = *long_count;
    for (uint32_t idx = blockIdx.x; idx < count; idx += gridDim.x) {
        sort_long_list((int)long_list[idx], ranges, depth_e, tile_keys, inst, gk, gv, s_sorted, s_run, s_e, S);
        __syncthreads();  // the LDS is reused by the next tile
    }
}


struct WsLayout {
    size_t vis_k0, vis_v0, inst_k2, inst_v2, depth_e, hist, sums, status, tickets, cnt, long_list, total;
    int64_t spine_tiles, n_status;
};

constexpr int kMaxPasses = 4;            // radix passes per sort (32-bit keys)
constexpr int kTickets = kMaxPasses + 1; // one per radix pass of the tile sort, then the long-list count

WsLayout ws_layout(int n, int n_views, int64_t capacity) {
    auto al = [](size_t x) { return (x + 255) & ~(size_t)255; };
    const int64_t vn = (int64_t)n * n_views;
    const int64_t cap = capacity > 0 ? capacity : 1;
    const int64_t big = vn > cap ? vn : cap;
    const int64_t nblk = rs_blocks(big);
    WsLayout L;
    L.spine_tiles = lb_tiles(256 * nblk);
    // run counts of the compaction, then tile totals of the instance-offset
    // scan (runs are the shorter, so there are more of them)
    const int64_t vt = (vn + CV_RUN - 1) / CV_RUN > 0 ? (vn + CV_RUN - 1) / CV_RUN : 1;
    static_assert(CV_RUN <= LB_TILE, "the run counts need at least as many words as the tile totals");
    // look-back status words: kMaxPasses radix spines
    L.n_status = kMaxPasses * L.spine_tiles;
    size_t o = 0;
    L.vis_k0 = o; o += al(4 * (size_t)(vn > 0 ? vn : 1));
    L.vis_v0 = o; o += al(4 * (size_t)(vn > 0 ? vn : 1));
    L.inst_k2 = o; o += al(4 * (size_t)cap);
    L.inst_v2 = o; o += al(4 * (size_t)cap);
    L.depth_e = o; o += al(4 * (size_t)cap);
    L.hist = o; o += al(4 * (size_t)(256 * nblk + 1));
    L.sums = o; o += al(4 * (size_t)vt);
    L.status = o; o += al(8 * (size_t)L.n_status);
    L.tickets = o; o += al(4 * (size_t)kTickets);
    L.cnt = o; o += al(8 * 4);
    // tiles with more than kTsShort instances: at most capacity / (kTsShort + 1)
    L.long_list = o; o += al(4 * (size_t)(cap / (kTsShort + 1) + 1));
    L.total = o;
    return L;
}

}  // namespace

size_t binsort_workspace_bytes(int n, int n_views, int64_t capacity) { return ws_layout(n, n_views, capacity).total; }

// Reads a look-back wait may take before it gives up (LB_SPIN_MAX, or the
// value of SGS_LOOKBACK_SPIN, which tests set to force the give-up path).
int lookback_spin_limit() {
    const char* v = std::getenv("SGS_LOOKBACK_SPIN");
    if (v == nullptr || *v == 0) return LB_SPIN_MAX;
    const long x = std::strtol(v, nullptr, 10);
    return x < 0 ? 0 : (x > LB_SPIN_MAX ? LB_SPIN_MAX : (int)x);
}

hipError_t launch_binsort(const uint32_t* rect, const int32_t* touched, int n,
                          const gs_view* views_dev, int n_views, int total_tiles, int tile, void* ws,
                          int64_t capacity, uint32_t* tile_keys, int32_t* inst, int32_t* inst_gid,
                          int32_t* pair_first, int32_t* ranges, int64_t* counts, hipStream_t s) {
    const WsLayout L = ws_layout(n, n_views, capacity);
    char* w = static_cast<char*>(ws);
    uint32_t* vis_k0 = reinterpret_cast<uint32_t*>(w + L.vis_k0);
    uint32_t* vis_v0 = reinterpret_cast<uint32_t*>(w + L.vis_v0);
    uint32_t* ik2 = reinterpret_cast<uint32_t*>(w + L.inst_k2);
    uint32_t* iv2 = reinterpret_cast<uint32_t*>(w + L.inst_v2);
    uint32_t* depth_e = reinterpret_cast<uint32_t*>(w + L.depth_e);
    uint32_t* hist = reinterpret_cast<uint32_t*>(w + L.hist);
    uint32_t* sums = reinterpret_cast<uint32_t*>(w + L.sums);
    uint64_t* status = reinterpret_cast<uint64_t*>(w + L.status);
    uint32_t* tickets = reinterpret_cast<uint32_t*>(w + L.tickets);
    int64_t* cnt = reinterpret_cast<int64_t*>(w + L.cnt);  // [0] n_vis [1] n_inst [2] clamped
    const int64_t vn = (int64_t)n * n_views;
    hipError_t e;

    // 0. zero the scan state and the counts, and clear the per-tile ranges
    hipLaunchKernelGGL(k_bin_reset, dim3(64), dim3(256), 0, s, status, L.n_status, tickets, kTickets,
                       reinterpret_cast<uint32_t*>(ranges), 2 * (int64_t)total_tiles);
    // 1. order-preserving compaction of the visible pairs: (tile count, pair)
    if (vn > 0) {
        const unsigned nrun = (unsigned)((vn + CV_RUN - 1) / CV_RUN);
        hipLaunchKernelGGL(k_count_visible, dim3(nrun), dim3(CV_THREADS), 0, s, touched, vn, sums);
        hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(TOP_THREADS), 0, s, sums, (int)nrun, &cnt[0]);
        hipLaunchKernelGGL(k_compact_visible, dim3(nrun), dim3(CV_THREADS), 0, s, touched, sums, vn, vis_k0, vis_v0);
    } else {
        e = fill_u32(reinterpret_cast<uint32_t*>(cnt), 0u, 8, s);
        if (e != hipSuccess) return e;
    }
    // 2. instance offsets in pair order (in place over the tile counts),
    //    total instance count and the counts
    e = exclusive_scan_long(LoadU32{vis_k0}, &cnt[0], vn, sums, vis_k0, &cnt[1], s,
                            CountsOut{counts, &cnt[2], &cnt[0], capacity});
    if (e != hipSuccess) return e;
    // 3. emission, then stable sort by global tile id
    int bits = 1;
    while ((1ll << bits) < (int64_t)total_tiles) ++bits;
    const int passes = (bits + 7) / 8;
    if (passes > kMaxPasses) return hipErrorInvalidValue;
    uint32_t* ek = (passes % 2 == 0) ? reinterpret_cast<uint32_t*>(tile_keys) : ik2;
    uint32_t* ev = (passes % 2 == 0) ? reinterpret_cast<uint32_t*>(inst) : iv2;
    uint32_t* ok = (passes % 2 == 0) ? ik2 : reinterpret_cast<uint32_t*>(tile_keys);
    uint32_t* ov = (passes % 2 == 0) ? iv2 : reinterpret_cast<uint32_t*>(inst);
    if (vn > 0) {
        hipLaunchKernelGGL(k_emit, dim3((unsigned)((vn + 255) / 256)), dim3(256), 0, s, vis_v0, vis_k0, &cnt[0],
                           reinterpret_cast<const uint4*>(rect), views_dev, n, tile, capacity, ek, inst_gid, depth_e,
                           pair_first);
    }
    // a look-back that waits past the spin limit (SGS_LOOKBACK_SPIN overrides
    // it, for tests) records the give-up in counts[3] and counts[4]
    LbGiveUp gu;
    gu.flag = reinterpret_cast<uint32_t*>(counts + 3);
    gu.sticky = reinterpret_cast<uint32_t*>(counts + 4);
    gu.spin_limit = lookback_spin_limit();
    e = radix_sort(ek, ev, ok, ov, &cnt[2], capacity, passes, hist, status, L.spine_tiles, tickets, gu, s);
    if (e != hipSuccess) return e;
    // 4. per-tile [start, end) (the ranges were cleared in step 0), then each
    //    tile's list in depth order
    if (capacity > 0) {
        hipLaunchKernelGGL(k_ranges, dim3((unsigned)((capacity + 255) / 256)), dim3(256), 0, s,
                           reinterpret_cast<const uint32_t*>(tile_keys), &cnt[2], reinterpret_cast<int2*>(ranges),
                           gu.flag);
        if (total_tiles > 0) {
            const int2* rg = reinterpret_cast<const int2*>(ranges);
            const int run = tile_run(tile);
            uint32_t* long_list = reinterpret_cast<uint32_t*>(w + L.long_list);
            uint32_t* long_count = tickets + kMaxPasses;
            hipLaunchKernelGGL(k_tile_sort_short, dim3(tile_grid(total_tiles, run)), dim3(TSS_THREADS), 0, s, rg,
                               total_tiles, run, depth_e, inst, long_list, long_count, gu.flag);
            const int64_t max_long = capacity / (kTsShort + 1) + 1;
            const unsigned lg = (unsigned)(max_long < 1024 ? max_long : 1024);
            hipLaunchKernelGGL(k_tile_sort_long, dim3(lg), dim3(TSL_THREADS), 0, s, rg, long_list, long_count,
                               depth_e, tile_keys, inst, ik2, iv2);
        }
    }
    return hipGetLastError();
}

}  // namespace sgs
