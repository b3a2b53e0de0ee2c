// k_sort.hip -- tile binning and global sort (Sec. 3.2 "Global Sorting and
// Tiling"): one (key, value) pair per touched tile, a stable LSD radix sort
// of the keys on the device, and the [start, end) range of every tile.
//
// key   = (global tile id << 32) | float32 bits of the centre's camera depth
// value = primitive index within its view
// Depths are beyond the near plane (> 0), so their float bits order like
// the depths themselves.  Pairs are emitted view by view, primitive by
// primitive, tiles row-major inside each primitive's rectangle; the sort is
// stable, so equal keys keep that order (ties go to the lower index).
#include "linprim_common.h"

namespace linprim {

__device__ inline void emit_pair(uint64_t g, uint32_t depth, uint32_t prim, uint32_t slot,
                                 uint64_t* __restrict__ keys, uint32_t* __restrict__ vals) {
    keys[slot] = (g << 32) | depth;
    vals[slot] = prim;
}

// One thread per (view, primitive) slot that touches a tile (from the
// scan's list, in slot order): one (key, value) pair per tile of the slot's
// tile rectangle, row-major, at the slot's offset.  The short runs (at most
// kShortRun tiles) of a wave's 64 slots are written together, one pair per
// lane and iteration: each lane finds the slot of its pair by a binary
// search over the wave's prefix of short-run lengths and takes the slot's
// rectangle from that lane; consecutive slots have consecutive offsets, so
// the stores are mostly contiguous.  Long runs (near or large primitives)
// are then written by the whole wave, one run at a time, and huge runs by
// the whole grid.
constexpr uint32_t kShortRun = 32;

__device__ inline void emit_wave(int64_t t, int64_t n_vis, const uint32_t* __restrict__ depth_keys,
                                 const uint32_t* __restrict__ tiles, const uint32_t* __restrict__ offsets,
                                 const uint2* __restrict__ trect, const ViewInfo* __restrict__ views,
                                 const uint32_t* __restrict__ vis, int64_t n,
                                 uint64_t* __restrict__ keys, uint32_t* __restrict__ vals) {
    const int lane = threadIdx.x & 63;
    uint32_t cnt = 0, key = 0, off = 0, prim = 0, ntx = 1, tiles_x = 0;
    uint64_t g0 = 0;                  // global tile of the rectangle's first tile
    if (t < n_vis) {
        const int64_t vs = vis[t];
        const int v = (int)(vs / n);
        prim = (uint32_t)(vs - (int64_t)v * n);
        cnt = tiles[vs];
        const uint2 tr = trect[vs];
        key = depth_keys[vs];
        off = offsets[vs];
        const int tx0 = (int)(tr.x & 0xffffu), ty0 = (int)(tr.x >> 16);
        ntx = tr.y & 0xffffu;
        const ViewInfo& V = views[v];
        tiles_x = (uint32_t)V.tiles_x;
        g0 = (uint64_t)(V.tile_base + (int64_t)ty0 * V.tiles_x + tx0);
    }
    // short runs: inclusive prefix of their lengths over the wave
    const uint32_t cs = cnt <= kShortRun ? cnt : 0u;
    uint32_t incl = wave_incl_scan_u32(cs);
    const uint32_t excl = incl - cs;
    const uint32_t total = (uint32_t)__builtin_amdgcn_readlane((int)incl, 63);
    for (uint32_t q = (uint32_t)lane; q - lane < total; q += 64) {
        // owner: the last lane whose exclusive prefix is <= q; a lane with an
        // empty or long run shares its prefix with the next lane, and lanes
        // at the end have prefix = total > q
        int lo = 0;
#pragma unroll
        for (int step = 32; step >= 1; step >>= 1) {
            const uint32_t e = (uint32_t)__shfl((int)excl, lo + step, 64);
            if (e <= q) lo += step;
        }
        const uint32_t r = q - (uint32_t)__shfl((int)excl, lo, 64);
        const uint32_t bo = (uint32_t)__shfl((int)off, lo, 64);
        const uint32_t bn = (uint32_t)__shfl((int)ntx, lo, 64);
        const uint32_t btx = (uint32_t)__shfl((int)tiles_x, lo, 64);
        const uint32_t bk = (uint32_t)__shfl((int)key, lo, 64);
        const uint32_t bp = (uint32_t)__shfl((int)prim, lo, 64);
        const uint64_t bg = ((uint64_t)(uint32_t)__shfl((int)(g0 >> 32), lo, 64) << 32) |
                            (uint32_t)__shfl((int)(uint32_t)g0, lo, 64);
        if (q < total) {
            const uint32_t row = r / bn, col = r - row * bn;
            const uint64_t g = bg + (uint64_t)row * btx + col;
            keys[bo + r] = (g << 32) | bk;
            vals[bo + r] = bp;
        }
    }
    // long runs: the whole wavefront writes each (huge ones are left to
    // the whole grid)
    uint64_t big = __ballot(cnt > kShortRun && cnt <= (uint32_t)kHugeRun);
    while (big) {
        const int b = __builtin_ctzll(big);
        big &= big - 1;
        const uint32_t c = (uint32_t)__builtin_amdgcn_readlane((int)cnt, b);
        const uint32_t o = (uint32_t)__builtin_amdgcn_readlane((int)off, b);
        const uint32_t k = (uint32_t)__builtin_amdgcn_readlane((int)key, b);
        const uint32_t pb = (uint32_t)__builtin_amdgcn_readlane((int)prim, b);
        const uint32_t bn = (uint32_t)__builtin_amdgcn_readlane((int)ntx, b);
        const uint32_t btx = (uint32_t)__builtin_amdgcn_readlane((int)tiles_x, b);
        const uint64_t bg = ((uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)(g0 >> 32), b) << 32) |
                            (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)g0, b);
        for (uint32_t q = (uint32_t)lane; q < c; q += 64) {
            const uint32_t row = q / bn, col = q - row * bn;
            keys[o + q] = ((bg + (uint64_t)row * btx + col) << 32) | k;
            vals[o + q] = pb;
        }
    }
}

__global__ __launch_bounds__(256) void k_emit_pairs(const uint32_t* __restrict__ depth_keys,
                                                    const uint32_t* __restrict__ tiles,
                                                    const uint32_t* __restrict__ offsets,
                                                    const uint2* __restrict__ trect,
                                                    const ViewInfo* __restrict__ views, const uint32_t* __restrict__ vis,
                                                    int64_t n, Status* __restrict__ status,
                                                    uint64_t capacity, const uint32_t* __restrict__ huge,
                                                    uint64_t* __restrict__ keys, uint32_t* __restrict__ vals,
                                                    uint2* __restrict__ ranges, int64_t n_tiles) {
    const int lane = threadIdx.x & 63;
    // the tile ranges start empty (k_tile_ranges fills them after the sort)
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n_tiles; t += (int64_t)gridDim.x * blockDim.x)
        ranges[t] = make_uint2(0u, 0u);
    if (blockIdx.x == 0 && threadIdx.x == 0) status->n_long = 0u;
    const uint64_t npairs = status->n_pairs;
    if (npairs > capacity) {
        if (blockIdx.x == 0 && threadIdx.x == 0) status->overflow = 1;
        return;
    }
    const int64_t n_vis = status->n_vis;
    // a grid of a few waves per CU strides over the list, 64 slots at a time
    const int64_t n_waves = (int64_t)gridDim.x * (blockDim.x >> 6);
    const int64_t wave_id = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    for (int64_t w0 = wave_id * 64; w0 < n_vis; w0 += n_waves * 64)
        emit_wave(w0 + lane, n_vis, depth_keys, tiles, offsets, trect, views, vis, n, keys, vals);
    // huge runs: 64-pair chunks dealt round-robin over all waves
    const uint32_t n_huge = status->n_huge;
    for (uint32_t i = 0; i < n_huge; ++i) {
        const int64_t vs = huge[i];
        const int v = (int)(vs / n);
        const uint32_t prim = (uint32_t)(vs - (int64_t)v * n);
        const uint32_t c = tiles[vs], o = offsets[vs], k = depth_keys[vs];
        const uint2 tr = trect[vs];
        const int tx0 = (int)(tr.x & 0xffffu), ty0 = (int)(tr.x >> 16);
        const uint32_t bn = tr.y & 0xffffu;
        const ViewInfo& V = views[v];
        const uint64_t bg = (uint64_t)(V.tile_base + (int64_t)ty0 * V.tiles_x + tx0);
        for (int64_t q0 = wave_id * 64; q0 < (int64_t)c; q0 += n_waves * 64) {
            const uint32_t q = (uint32_t)q0 + (uint32_t)lane;
            if (q < c) {
                const uint32_t row = q / bn, col = q - row * bn;
                keys[o + q] = ((bg + (uint64_t)row * (uint32_t)V.tiles_x + col) << 32) | k;
                vals[o + q] = prim;
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Per-tile sort (default).  A stable LSD radix sort of the tile bits alone
// (bits 32 and up of the keys) groups the pairs by tile and keeps each
// tile's pairs in emission order; each tile's list is then sorted by
// (depth bits, primitive index), which is unique within a tile, so the
// result is the order of the stable sort of the full keys.  Lists of up to
// kShortList entries are sorted by one wave (up to 64 by counting ranks,
// more by a bitonic network in registers); longer ones are sorted in LDS by
// a 256-thread block (bitonic network), and lists longer than kLdsList are
// sorted in kLdsList chunks that are then merged.
// ---------------------------------------------------------------------------
constexpr int kShortList = 512;
constexpr int kLdsList = 4096;

// Writes the sorted pair e of tile g: the full key and the value.
__device__ inline void put_sorted(uint64_t g, uint64_t dkey, uint32_t e, uint64_t* __restrict__ keys,
                                  uint32_t* __restrict__ vals) {
    keys[e] = (g << 32) | (dkey >> 32);
    vals[e] = (uint32_t)dkey;
}

// (depth bits, primitive index) of tile-sorted pair e.
__device__ inline uint64_t depth_index(const uint64_t* __restrict__ keys, const uint32_t* __restrict__ vals,
                                       int64_t e) {
    return ((uint64_t)(uint32_t)keys[e] << 32) | vals[e];
}

// Sorts the (depth, index) keys of a list of up to 64 P pairs with one wave:
// element e = 64 q + lane in register q (padded with ~0, which sorts last),
// a bitonic network whose partners in other lanes come by shuffles and whose
// partners in other registers of the lane are compared in place.
template <int P>
__device__ inline void bitonic_list(uint64_t (&k)[P], int lane) {
    constexpr int N = 64 * P;
#pragma unroll
    for (int size = 2; size <= N; size <<= 1) {
#pragma unroll
        for (int j = size >> 1; j >= 1; j >>= 1) {
            if (j >= 64) {
                const int qj = j >> 6;
#pragma unroll
                for (int q = 0; q < P; ++q) {
                    if (q & qj) continue;   // q holds the lower element of the pair
                    const bool up = ((q * 64 + lane) & size) == 0;
                    const uint64_t a = k[q], b = k[q | qj];
                    const bool sw = up ? (a > b) : (a < b);
                    k[q] = sw ? b : a;
                    k[q | qj] = sw ? a : b;
                }
            } else {
#pragma unroll
                for (int q = 0; q < P; ++q) {
                    const int e = q * 64 + lane;
                    const uint64_t a = k[q];
                    const uint32_t lo = (uint32_t)__shfl_xor((int)(uint32_t)a, j, 64);
                    const uint32_t hi = (uint32_t)__shfl_xor((int)(uint32_t)(a >> 32), j, 64);
                    const uint64_t b = ((uint64_t)hi << 32) | lo;
                    const bool keep_min = ((e & size) == 0) == ((e & j) == 0);
                    const bool a_min = a < b;
                    k[q] = (keep_min == a_min) ? a : b;
                }
            }
        }
    }
}

// A list of 64 < len <= 64 P pairs sorted by one wave (bitonic_list) and
// written back with its full keys.
template <int P>
__device__ inline void sort_list(const uint64_t* __restrict__ in_keys, const uint32_t* __restrict__ in_vals, uint2 rg,
                                 int len, int lane, uint64_t g, uint64_t* __restrict__ keys,
                                 uint32_t* __restrict__ vals) {
    uint64_t k[P];
#pragma unroll
    for (int q = 0; q < P; ++q) {
        const int e = q * 64 + lane;
        k[q] = (e < len) ? depth_index(in_keys, in_vals, rg.x + e) : ~0ull;
    }
    bitonic_list<P>(k, lane);
#pragma unroll
    for (int q = 0; q < P; ++q)
        if (q * 64 + lane < len) put_sorted(g, k[q], rg.x + q * 64 + lane, keys, vals);
}

// One wave per tile with at most kShortList pairs: up to 64 pairs, every
// pair's rank is the number of smaller (depth, index) values in the list;
// more, a bitonic sort in registers.  Longer lists are put on the long-list
// list.  Wave w takes the tile at position w of the backward render order
// (longest lists first, written just before).
__global__ __launch_bounds__(64) void k_sort_short_lists(const uint2* __restrict__ ranges, int64_t n_tiles,
                                                         Status* __restrict__ status, uint64_t capacity,
                                                         const uint64_t* __restrict__ in_keys,
                                                         const uint32_t* __restrict__ in_vals,
                                                         uint64_t* __restrict__ keys, uint32_t* __restrict__ vals,
                                                         uint32_t* __restrict__ long_list,
                                                         const uint32_t* __restrict__ order) {
    constexpr int PER = kShortList / 64;
    if (status->n_pairs > capacity) return;
    if ((int64_t)blockIdx.x >= n_tiles) return;
    // longest lists first, so that their sorts start first
    const int64_t g = order[blockIdx.x];
    const uint2 rg = ranges[g];
    const int len = (int)(rg.y - rg.x);
    if (len == 0) return;
    const int lane = threadIdx.x;
    if (len > kShortList) {
        if (lane == 0) long_list[atomicAdd(&status->n_long, 1u)] = (uint32_t)g;
        return;
    }
    if (len <= 64) {
        // one pair per lane
        const uint64_t k = (lane < len) ? depth_index(in_keys, in_vals, rg.x + lane) : ~0ull;
        uint32_t rank = 0;
        for (int j = 0; j < len; ++j) {
            const uint64_t kj = ((uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)(k >> 32), j) << 32) |
                                (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)k, j);
            rank += (kj < k) ? 1u : 0u;
        }
        if (lane < len) put_sorted((uint64_t)g, k, rg.x + rank, keys, vals);
        return;
    }
    if (len <= 128) sort_list<2>(in_keys, in_vals, rg, len, lane, (uint64_t)g, keys, vals);
    else if (len <= 256) sort_list<4>(in_keys, in_vals, rg, len, lane, (uint64_t)g, keys, vals);
    else sort_list<PER>(in_keys, in_vals, rg, len, lane, (uint64_t)g, keys, vals);
}

__device__ inline uint64_t shfl_xor_u64(uint64_t v, int m) {
    const uint32_t lo = (uint32_t)__shfl_xor((int)(uint32_t)v, m, 64);
    const uint32_t hi = (uint32_t)__shfl_xor((int)(uint32_t)(v >> 32), m, 64);
    return ((uint64_t)hi << 32) | lo;
}

// Bitonic sort of s[0, P) ascending, P a power of two in [128, kLdsList],
// by the whole block.  Compare-exchange steps whose partners are 64 or more
// apart go through LDS, one barrier each; the steps below 64 of every merge
// run in registers with shuffles (thread t holds elements t + blockDim m,
// whose partners then belong to lanes of the same wave).
__device__ inline void lds_bitonic(uint64_t* s, int P) {
    const int t = threadIdx.x, T = blockDim.x;
    for (int k = 2; k <= P; k <<= 1) {
        int j = k >> 1;
        for (; j >= 64; j >>= 1) {
            for (int i = t; i < (P >> 1); i += T) {
                const int lo = 2 * j * (i / j) + (i % j), hi = lo + j;
                const uint64_t a = s[lo], b = s[hi];
                const bool up = (lo & k) == 0;
                if ((a > b) == up) {
                    s[lo] = b;
                    s[hi] = a;
                }
            }
            __syncthreads();
        }
        // steps j < 64 (wave-uniform: P and T are multiples of 64)
        for (int e = t; e < P; e += T) {
            uint64_t v = s[e];
            const bool up = (e & k) == 0;
            for (int jj = j; jj > 0; jj >>= 1) {
                const uint64_t o = shfl_xor_u64(v, jj);
                const bool keep_min = ((e & jj) == 0) == up;
                v = keep_min ? (o < v ? o : v) : (o > v ? o : v);
            }
            s[e] = v;
        }
        __syncthreads();
    }
}

// Merge of the sorted runs a[0, la) and b[0, lb) into out[0, la + lb) by the
// whole block: thread t produces a contiguous slice of the output, finding
// where it starts by a binary search on the merge path.
__device__ inline void block_merge(const uint64_t* __restrict__ a, int64_t la, const uint64_t* __restrict__ b,
                                   int64_t lb, uint64_t* __restrict__ out) {
    const int64_t m = la + lb;
    const int64_t per = (m + blockDim.x - 1) / blockDim.x;
    const int64_t d0 = min(m, (int64_t)threadIdx.x * per), d1 = min(m, d0 + per);
    if (d0 >= d1) return;
    // smallest i with a[i] > b[d0 - i - 1] (keys are unique)
    int64_t lo = max((int64_t)0, d0 - lb), hi = min(d0, la);
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (a[mid] < b[d0 - mid - 1]) lo = mid + 1; else hi = mid;
    }
    int64_t i = lo, j = d0 - lo;
    for (int64_t d = d0; d < d1; ++d) {
        const bool take_a = j >= lb || (i < la && a[i] < b[j]);
        out[d] = take_a ? a[i++] : b[j++];
    }
}

// Tiles with more than kShortList pairs, one block at a time.  The (depth,
// index) values are formed in place of the tile-sorted keys, which are no
// longer needed, and merged through the output key array.
__global__ __launch_bounds__(256) void k_sort_long_lists(const uint2* __restrict__ ranges,
                                                         const uint32_t* __restrict__ long_list,
                                                         const Status* __restrict__ status, uint64_t capacity,
                                                         uint64_t* __restrict__ in_keys,
                                                         const uint32_t* __restrict__ in_vals,
                                                         uint64_t* __restrict__ keys, uint32_t* __restrict__ vals) {
    __shared__ uint64_t s[kLdsList];
    if (status->n_pairs > capacity) return;
    const uint32_t n_long = status->n_long;
    for (uint32_t li = blockIdx.x; li < n_long; li += gridDim.x) {
        const uint64_t g = long_list[li];
        const uint2 rg = ranges[g];
        const int64_t len = (int64_t)rg.y - rg.x;
        uint64_t* seg = in_keys + rg.x;
        if (len <= kLdsList) {
            // one chunk: sorted in LDS and written out from there
            int P = 128;
            while (P < len) P <<= 1;
            for (int i = threadIdx.x; i < P; i += blockDim.x)
                s[i] = (i < len) ? depth_index(in_keys, in_vals, (int64_t)rg.x + i) : ~0ull;
            __syncthreads();
            lds_bitonic(s, P);
            for (int i = threadIdx.x; i < len; i += blockDim.x) put_sorted(g, s[i], rg.x + (uint32_t)i, keys, vals);
            __syncthreads();
            continue;
        }
        // sort chunks of kLdsList in LDS, written back in place
        for (int64_t c0 = 0; c0 < len; c0 += kLdsList) {
            const int cl = (int)min((int64_t)kLdsList, len - c0);
            int P = 128;
            while (P < cl) P <<= 1;
            for (int i = threadIdx.x; i < P; i += blockDim.x)
                s[i] = (i < cl) ? depth_index(in_keys, in_vals, (int64_t)rg.x + c0 + i) : ~0ull;
            __syncthreads();
            lds_bitonic(s, P);
            for (int i = threadIdx.x; i < cl; i += blockDim.x) seg[c0 + i] = s[i];
            __syncthreads();
        }
        // merge runs of doubling width, ping-ponging between the segment and
        // the output key array's segment (scratch until the final write)
        uint64_t* src = seg;
        uint64_t* dst = keys + rg.x;
        for (int64_t w = kLdsList; w < len; w <<= 1) {
            for (int64_t a0 = 0; a0 < len; a0 += 2 * w) {
                const int64_t la = min(w, len - a0), lb = min(w, len - a0 - la);
                block_merge(src + a0, la, src + a0 + la, lb, dst + a0);
            }
            __syncthreads();
            uint64_t* sw = src; src = dst; dst = sw;
        }
        // src holds the sorted list; each index is read and then written by
        // the same thread
        for (int64_t i = threadIdx.x; i < len; i += blockDim.x) put_sorted(g, src[i], rg.x + (uint32_t)i, keys, vals);
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// LSD radix sort, one pass per digit of `bits` bits starting at `shift`.
// Each block owns kSortTile consecutive keys.
//   1) k_radix_hist: per-block digit histogram -> hist[digit][block]
//   2) k_radix_scan: per digit, exclusive prefix over blocks (in place) and
//      the digit total
//   3) k_radix_scatter: stable rank inside the block, plus the digit's base
//      and the block's prefix -> output position
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kSortThreads) void k_radix_hist(const uint64_t* __restrict__ keys,
                                                             const Status* __restrict__ status, uint64_t capacity,
                                                             int shift, int bits, int64_t nblocks,
                                                             uint32_t* __restrict__ hist) {
    __shared__ uint32_t h[256];
    const uint64_t np = status->n_pairs;
    if (np > capacity) return;
    const int radix = 1 << bits;
    for (int d = threadIdx.x; d < radix; d += kSortThreads) h[d] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * kSortTile;
    for (int k = 0; k < kSortItems; ++k) {
        const int64_t idx = base + (int64_t)k * kSortThreads + threadIdx.x;
        if (idx < (int64_t)np) {
            const uint32_t d = (uint32_t)(keys[idx] >> shift) & (uint32_t)(radix - 1);
            atomicAdd(&h[d], 1u);
        }
    }
    __syncthreads();
    for (int d = threadIdx.x; d < radix; d += kSortThreads) hist[(int64_t)d * nblocks + blockIdx.x] = h[d];
}

// One block per digit: exclusive prefix of the digit's per-block counts over
// the blocks (in place), 1024 at a time (wave scans by shuffles, then the
// wave totals), and the digit's total.
__global__ __launch_bounds__(1024) void k_radix_scan(uint32_t* __restrict__ hist, const Status* __restrict__ status,
                                                     uint64_t capacity, int64_t nblocks,
                                                     uint32_t* __restrict__ digit_totals) {
    __shared__ uint32_t wsum[16];
    if (status->n_pairs > capacity) return;
    const int d = blockIdx.x;
    uint32_t* row = hist + (int64_t)d * nblocks;
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    uint32_t carry = 0;
    for (int64_t b0 = 0; b0 < nblocks; b0 += 1024) {
        const int64_t idx = b0 + t;
        const uint32_t x = (idx < nblocks) ? row[idx] : 0u;
        uint32_t incl = wave_incl_scan_u32(x);
        if (lane == 63) wsum[wave] = incl;
        __syncthreads();
        uint32_t before = 0, total = 0;
#pragma unroll
        for (int w = 0; w < 16; ++w) {
            const uint32_t v = wsum[w];
            before += (w < wave) ? v : 0u;
            total += v;
        }
        if (idx < nblocks) row[idx] = carry + before + incl - x;
        carry += total;
        __syncthreads();
    }
    if (t == 0) digit_totals[d] = carry;
}

__global__ __launch_bounds__(kSortThreads) void k_radix_scatter(const uint64_t* __restrict__ keys_in,
                                                                const uint32_t* __restrict__ vals_in,
                                                                const Status* __restrict__ status, uint64_t capacity,
                                                                int shift, int bits, int64_t nblocks,
                                                                const uint32_t* __restrict__ hist,
                                                                const uint32_t* __restrict__ digit_totals,
                                                                uint64_t* __restrict__ keys_out,
                                                                uint32_t* __restrict__ vals_out) {
    constexpr int NW = kSortThreads / 64;
    __shared__ uint32_t base[256];       // global start of each digit for this block
    __shared__ uint32_t running[256];    // keys of each digit in this block
    __shared__ uint32_t dstart[256];     // first position of each digit in lkey
    // keys of each digit per (item round, wave), then their exclusive prefix
    // over the rounds and waves in index order
    __shared__ uint32_t cnt[kSortItems][NW][256];
    __shared__ uint64_t lkey[kSortTile];  // the block's keys in digit order
    __shared__ uint32_t lval[kSortTile];
    const uint64_t np = status->n_pairs;
    if (np > capacity) return;
    const int radix = 1 << bits;
    const int t = threadIdx.x;
    const int wave = t >> 6, lane = t & 63;
    // digit bases: exclusive scan of the digit totals (one wave), plus this
    // block's prefix within the digit
    if (t < 64) {
        uint32_t carry = 0;
        for (int d0 = 0; d0 < radix; d0 += 64) {
            const int d = d0 + lane;
            uint32_t x = (d < radix) ? digit_totals[d] : 0u;
            uint32_t incl = wave_incl_scan_u32(x);
            if (d < radix) base[d] = carry + incl - x + hist[(int64_t)d * nblocks + blockIdx.x];
            carry += (uint32_t)__builtin_amdgcn_readlane((int)incl, 63);
        }
    }
    for (int d = t; d < 256; d += kSortThreads)
        for (int k = 0; k < kSortItems; ++k)
            for (int w = 0; w < NW; ++w) cnt[k][w][d] = 0;
    __syncthreads();
    // 1. rank of every key among the block's keys of its digit, in index order
    const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    const int64_t blk = (int64_t)blockIdx.x * kSortTile;
    uint64_t key[kSortItems];
    uint32_t val[kSortItems], dig[kSortItems], rnk[kSortItems];
#pragma unroll
    for (int k = 0; k < kSortItems; ++k) {
        const int64_t idx = blk + (int64_t)k * kSortThreads + t;
        const bool valid = idx < (int64_t)np;
        key[k] = valid ? keys_in[idx] : 0ull;
        val[k] = valid ? vals_in[idx] : 0u;
    }
#pragma unroll
    for (int k = 0; k < kSortItems; ++k) {
        const int64_t idx = blk + (int64_t)k * kSortThreads + t;
        const bool valid = idx < (int64_t)np;
        const uint32_t d = valid ? (uint32_t)(key[k] >> shift) & (uint32_t)(radix - 1) : 0u;
        dig[k] = d;
        // lanes of this wave holding the same digit
        uint64_t peers = __ballot(valid);
        for (int b = 0; b < bits; ++b) {
            const uint64_t m = __ballot(valid && ((d >> b) & 1u));
            peers &= ((d >> b) & 1u) ? m : ~m;
        }
        const uint32_t rank = (uint32_t)__popcll(peers & lt_mask);
        if (valid && rank == 0) cnt[k][wave][d] = (uint32_t)__popcll(peers);
        rnk[k] = rank;
    }
    __syncthreads();
    // per digit: exclusive prefix over (round, wave) in index order
    for (int d = t; d < radix; d += kSortThreads) {
        uint32_t run = 0;
        for (int k = 0; k < kSortItems; ++k)
            for (int w = 0; w < NW; ++w) {
                const uint32_t c = cnt[k][w][d];
                cnt[k][w][d] = run;
                run += c;
            }
        running[d] = run;
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kSortItems; ++k) rnk[k] += cnt[k][wave][dig[k]];
    // 2. the block's digit starts (exclusive scan of its digit counts, one
    //    wave), keys placed in LDS in digit order
    if (t < 64) {
        uint32_t carry = 0;
        for (int d0 = 0; d0 < radix; d0 += 64) {
            const int d = d0 + lane;
            const uint32_t x = (d < radix) ? running[d] : 0u;
            uint32_t incl = wave_incl_scan_u32(x);
            if (d < radix) dstart[d] = carry + incl - x;
            carry += (uint32_t)__builtin_amdgcn_readlane((int)incl, 63);
        }
    }
    __syncthreads();
    const int nk = (int)min((int64_t)kSortTile, (int64_t)np - blk);
#pragma unroll
    for (int k = 0; k < kSortItems; ++k) {
        const int64_t idx = blk + (int64_t)k * kSortThreads + t;
        if (idx < (int64_t)np) {
            const uint32_t lp = dstart[dig[k]] + rnk[k];
            lkey[lp] = key[k];
            lval[lp] = val[k];
        }
    }
    __syncthreads();
    // 3. consecutive threads write consecutive positions of each digit's run
    for (int i = t; i < nk; i += kSortThreads) {
        const uint64_t kk = lkey[i];
        const uint32_t d = (uint32_t)(kk >> shift) & (uint32_t)(radix - 1);
        const uint32_t pos = base[d] + (uint32_t)i - dstart[d];
        keys_out[pos] = kk;
        vals_out[pos] = lval[i];
    }
}

__global__ __launch_bounds__(256) void k_clear_ranges(uint2* __restrict__ ranges, int64_t count,
                                                      Status* __restrict__ status) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) ranges[i] = make_uint2(0u, 0u);
    if (i == 0) status->n_long = 0u;
}

__global__ __launch_bounds__(256) void k_tile_ranges(const uint64_t* __restrict__ keys,
                                                     const Status* __restrict__ status, uint64_t capacity,
                                                     uint2* __restrict__ ranges) {
    const uint64_t np = status->n_pairs;
    if (np > capacity) return;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (int64_t)np) return;
    const uint32_t tile = (uint32_t)(keys[i] >> 32);
    if (i == 0 || (uint32_t)(keys[i - 1] >> 32) != tile) ranges[tile].x = (uint32_t)i;
    if (i == (int64_t)np - 1 || (uint32_t)(keys[i + 1] >> 32) != tile) ranges[tile].y = (uint32_t)(i + 1);
}

// Render orders.  The backward (and the exact variant's forward) takes the
// tiles by list length, longest first, in kOrderClasses classes (tile order
// inside a class), so that the waves that start last are short.  The
// ray-space forward, whose walks are cheaper and more sensitive to cache
// locality, takes them in kFwdGroups coarser groups of consecutive classes
// (tile order inside a group).  Counts are kept class-major, sums[c *
// nblocks + b] for class c in block b of `items` tiles (order_items), so that
// one exclusive scan over them gives every (class, block) its first position.
__device__ inline int order_class(uint32_t len) {
    int c = 0;
#pragma unroll
    for (int k = 0; k < kOrderClasses - 1; ++k) c += (len <= kOrderBounds[k]) ? 1 : 0;
    return c;
}

__global__ __launch_bounds__(256) void k_order_count(const uint2* __restrict__ ranges, int64_t n_tiles,
                                                     const Status* __restrict__ status, uint64_t capacity,
                                                     uint32_t* __restrict__ sums, int items) {
    __shared__ uint32_t cnt[kOrderClasses];
    if (status->n_pairs > capacity) return;
    if (threadIdx.x < kOrderClasses) cnt[threadIdx.x] = 0u;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * items;
    for (int k = 0; k < items / 256; ++k) {
        const int64_t g = base + k * 256 + threadIdx.x;
        if (g < n_tiles) {
            const uint2 rg = ranges[g];
            atomicAdd(&cnt[order_class(rg.y - rg.x)], 1u);
        }
    }
    __syncthreads();
    if (threadIdx.x < kOrderClasses) sums[(int64_t)threadIdx.x * gridDim.x + blockIdx.x] = cnt[threadIdx.x];
}

// Many blocks: one block turns the count entries into exclusive prefixes in
// place, the total after them.
__global__ __launch_bounds__(1024) void k_order_prefix(uint32_t* __restrict__ sums, int64_t count,
                                                       const Status* __restrict__ status, uint64_t capacity) {
    __shared__ uint32_t wsum[16];
    if (status->n_pairs > capacity) return;
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    uint32_t carry = 0;
    for (int64_t b0 = 0; b0 < count; b0 += 1024) {
        const int64_t idx = b0 + t;
        const uint32_t x = (idx < count) ? sums[idx] : 0u;
        uint32_t incl = wave_incl_scan_u32(x);
        if (lane == 63) wsum[wave] = incl;
        __syncthreads();
        uint32_t wb = 0, tot = 0;
#pragma unroll
        for (int w = 0; w < 16; ++w) {
            wb += (w < wave) ? wsum[w] : 0u;
            tot += wsum[w];
        }
        if (idx < count) sums[idx] = carry + wb + incl - x;
        carry += tot;
        __syncthreads();
    }
    if (t == 0) sums[count] = carry;
}

// Backward order: tile g of class c goes to (first position of c in this
// block) + (tiles of class c before g in this block).  Forward order: the
// same with groups of consecutive classes in place of the classes.  The
// block takes its tiles in rounds of 256, in tile order; a tile's rank among
// the tiles of its wave with the same class (or group) comes from ballots.
// Counter slots: classes 0..K-1, then groups K..K+G-1; first[K + G + g] is
// the first position of group g in the whole forward order.
static_assert(kOrderDirectBlocks <= 256, "direct mode: one block's counts per thread");

// Sum over the 64 lanes of a wave by DPP steps (every lane must be active);
// lane 63 ends with the total, which is returned to every lane.
__device__ inline uint32_t wave_sum_u32(uint32_t v) {
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0xB1, 0xF, 0xF, false);    // quad_perm(1,0,3,2)
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x4E, 0xF, 0xF, false);    // quad_perm(2,3,0,1)
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x141, 0xF, 0xF, false);   // row_half_mirror
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x140, 0xF, 0xF, false);   // row_mirror
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x142, 0xA, 0xF, false);   // row_bcast:15
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x143, 0x8, 0xF, false);   // row_bcast:31
    return (uint32_t)__builtin_amdgcn_readlane((int)v, 63);
}

__device__ inline int order_group(int c) {
    int g = 0;
#pragma unroll
    for (int k = 0; k < kFwdGroups - 1; ++k) g += (c > kFwdGroupLast[k]) ? 1 : 0;
    return g;
}

__global__ __launch_bounds__(256) void k_order_write(const uint2* __restrict__ ranges, int64_t n_tiles,
                                                     const Status* __restrict__ status, uint64_t capacity,
                                                     const uint32_t* __restrict__ sums, int64_t nblocks,
                                                     bool prefixed, uint32_t* __restrict__ order_fwd,
                                                     uint32_t* __restrict__ order_bwd, int items) {
    constexpr int K = kOrderClasses, G = kFwdGroups, NS = K + G;
    __shared__ uint32_t first[NS + G];
    __shared__ uint32_t running[NS];
    __shared__ uint32_t wave_cnt[4][NS + G];
    if (status->n_pairs > capacity) return;
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int64_t b = blockIdx.x;
    if (prefixed) {
        // sums holds the exclusive scan: the first position of class c is
        // sums[c nblocks], its tiles in the blocks before b sums[c nblocks + b]
        // - sums[c nblocks]
        if (t < K) first[t] = sums[(int64_t)t * nblocks + b];
        if (t >= K && t < NS) {
            const int g = t - K;
            uint32_t v = 0;
            for (int c = (g == 0) ? 0 : kFwdGroupLast[g - 1] + 1; c <= kFwdGroupLast[g]; ++c)
                v += sums[(int64_t)c * nblocks + b] - sums[(int64_t)c * nblocks];
            first[t] = v;
        }
        if (t >= NS && t < NS + G) {
            const int g = t - NS;
            first[t] = sums[(int64_t)((g == 0) ? 0 : kFwdGroupLast[g - 1] + 1) * nblocks];
        }
    } else {
        // thread t < nblocks reads block t's counts: first[c] sums the counts
        // of the classes before c in all blocks and of class c in the blocks
        // before b; then the tiles of each group in the blocks before b; then
        // the tiles of the classes before each group
        uint32_t part[NS + G];
#pragma unroll
        for (int c = 0; c < NS + G; ++c) part[c] = 0u;
        if (t < nblocks) {
            const bool before = t < b;
            uint32_t acc = 0;
#pragma unroll
            for (int c = 0; c < K; ++c) {
                const uint32_t x = sums[(int64_t)c * nblocks + t];
                const int g = order_group(c);
                if (c == 0 || order_group(c - 1) != g) part[NS + g] = acc;
                part[c] = acc + (before ? x : 0u);
                part[K + g] += before ? x : 0u;
                acc += x;
            }
        }
#pragma unroll
        for (int c = 0; c < NS + G; ++c) {
            const uint32_t v = wave_sum_u32(part[c]);
            if (lane == 0) wave_cnt[wave][c] = v;
        }
        __syncthreads();
        if (t < NS + G) first[t] = wave_cnt[0][t] + wave_cnt[1][t] + wave_cnt[2][t] + wave_cnt[3][t];
        __syncthreads();
    }
    if (t < NS) running[t] = 0u;
    const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    for (int r = 0; r < items / 256; ++r) {
        const int64_t g = b * items + r * 256 + t;
        const bool valid = g < n_tiles;
        int c = 0;
        if (valid) {
            const uint2 rg = ranges[g];
            c = order_class(rg.y - rg.x);
        }
        uint64_t peers = __ballot(valid);
#pragma unroll
        for (int bit = 0; bit < 4; ++bit) {
            const uint64_t m = __ballot(valid && ((c >> bit) & 1));
            peers &= ((c >> bit) & 1) ? m : ~m;
        }
        const int grp = order_group(c);
        uint64_t gm = 0;   // lanes of this wave in the tile's group
#pragma unroll
        for (int k = 0; k < G; ++k) {
            const uint64_t m = __ballot(valid && grp == k);
            if (lane == 0) wave_cnt[wave][K + k] = (uint32_t)__popcll(m);
            gm = (grp == k) ? m : gm;
        }
        if (lane < K) wave_cnt[wave][lane] = 0u;
        const uint32_t rank = (uint32_t)__popcll(peers & lt_mask);
        if (valid && rank == 0) wave_cnt[wave][c] = (uint32_t)__popcll(peers);
        __syncthreads();
        if (valid) {
            const int s = K + grp;
            uint32_t pos = first[c] + running[c] + rank;
            uint32_t pf = first[NS + grp] + first[s] + running[s] + (uint32_t)__popcll(gm & lt_mask);
            for (int w = 0; w < wave; ++w) {
                pos += wave_cnt[w][c];
                pf += wave_cnt[w][s];
            }
            order_bwd[pos] = (uint32_t)g;
            order_fwd[pf] = (uint32_t)g;
        }
        __syncthreads();
        if (t < NS) running[t] += wave_cnt[0][t] + wave_cnt[1][t] + wave_cnt[2][t] + wave_cnt[3][t];
        __syncthreads();
    }
}

// Passes over the tile bits alone (per-tile sort): at most 8 bits each,
// spread evenly.
inline void tile_passes(int tile_bits, int* passes, int* digit) {
    *passes = (tile_bits + 7) / 8;
    *digit = (tile_bits + *passes - 1) / *passes;
}

int sorted_buffer(int64_t n_tiles_total, bool radix, int digit_bits) {
    const int tb = key_tile_bits(n_tiles_total);
    if (radix) return ((32 + tb + digit_bits - 1) / digit_bits) & 1;
    int passes, digit;
    tile_passes(tb, &passes, &digit);
    return (passes & 1) ^ 1;   // the per-list sort writes to the other buffer
}

hipError_t launch_bin_sort(const ViewLayout& L, char* vws, const PairLayout& P, char* pws, bool radix, int tile,
                           int digit_bits, int32_t n_views, const linprim_camera* cams, hipStream_t stream,
                           int* result_in_b) {
    (void)cams;
    const int shift = (tile == 8) ? 3 : (tile == 16) ? 4 : 5;
    Status* status = reinterpret_cast<Status*>(vws + L.status);
    const ViewInfo* views = reinterpret_cast<const ViewInfo*>(vws + L.views);
    uint64_t* ka = reinterpret_cast<uint64_t*>(pws + P.keys_a);
    uint64_t* kb = reinterpret_cast<uint64_t*>(pws + P.keys_b);
    uint32_t* va = reinterpret_cast<uint32_t*>(pws + P.vals_a);
    uint32_t* vb = reinterpret_cast<uint32_t*>(pws + P.vals_b);
    uint32_t* hist = reinterpret_cast<uint32_t*>(pws + P.hist);
    uint32_t* totals = hist + (int64_t)256 * P.sort_blocks;
    uint2* ranges = reinterpret_cast<uint2*>(vws + L.ranges);
    uint32_t* long_list = reinterpret_cast<uint32_t*>(vws + L.long_list);
    const uint64_t cap = (uint64_t)P.capacity;
    const int64_t nt = L.n_tiles_total;
    if (L.n > 0) {
        const int64_t vn = L.n * (int64_t)n_views;
        // enough 4-wave blocks for the list, at most 2048 (32 waves per CU)
        const int64_t blocks = (vn + 255) / 256 < 2048 ? (vn + 255) / 256 : 2048;
        hipLaunchKernelGGL(k_emit_pairs, dim3((unsigned)blocks), dim3(256), 0, stream,
                           reinterpret_cast<const uint32_t*>(vws + L.depth_keys),
                           reinterpret_cast<const uint32_t*>(vws + L.tiles),
                           reinterpret_cast<const uint32_t*>(vws + L.offsets),
                           reinterpret_cast<const uint2*>(vws + L.trect), views,
                           reinterpret_cast<const uint32_t*>(vws + L.vis), L.n, status, cap,
                           reinterpret_cast<const uint32_t*>(vws + L.huge), ka, va, ranges, nt);
    } else {
        hipLaunchKernelGGL(k_clear_ranges, dim3((unsigned)((nt + 255) / 256)), dim3(256), 0, stream, ranges, nt,
                           status);
    }
    const int tb = key_tile_bits(nt);
    int passes, digit, key_lo, key_bits;
    if (radix) {
        key_lo = 0;
        key_bits = 32 + tb;
        digit = digit_bits;
        passes = (key_bits + digit - 1) / digit;
    } else {
        key_lo = 32;
        key_bits = tb;
        tile_passes(tb, &passes, &digit);
    }
    uint64_t *kin = ka, *kout = kb;
    uint32_t *vin = va, *vout = vb;
    const int64_t nb = P.sort_blocks;
    for (int p = 0; p < passes; ++p) {
        const int sh = p * digit;
        const int bits = (key_bits - sh) < digit ? (key_bits - sh) : digit;
        if (nb > 0) {
            hipLaunchKernelGGL(k_radix_hist, dim3((unsigned)nb), dim3(kSortThreads), 0, stream, kin, status, cap,
                               key_lo + sh, bits, nb, hist);
            hipLaunchKernelGGL(k_radix_scan, dim3(1u << bits), dim3(1024), 0, stream, hist, status, cap, nb, totals);
            hipLaunchKernelGGL(k_radix_scatter, dim3((unsigned)nb), dim3(kSortThreads), 0, stream, kin, vin, status,
                               cap, key_lo + sh, bits, nb, hist, totals, kout, vout);
        }
        uint64_t* tk = kin; kin = kout; kout = tk;
        uint32_t* tv = vin; vin = vout; vout = tv;
    }
    if (P.capacity > 0)
        hipLaunchKernelGGL(k_tile_ranges, dim3((unsigned)((P.capacity + 255) / 256)), dim3(256), 0, stream, kin, status,
                           cap, ranges);
    {
        uint32_t* order = reinterpret_cast<uint32_t*>(vws + L.order);
        uint32_t* order_bwd = reinterpret_cast<uint32_t*>(vws + L.order_bwd);
        uint32_t* osums = reinterpret_cast<uint32_t*>(vws + L.order_sums);
        const int items = order_items(nt);
        const int64_t ob = (nt + items - 1) / items;
        hipLaunchKernelGGL(k_order_count, dim3((unsigned)ob), dim3(256), 0, stream, ranges, nt, status, cap, osums,
                           items);
        const bool prefixed = ob > kOrderDirectBlocks;
        if (prefixed)
            hipLaunchKernelGGL(k_order_prefix, dim3(1), dim3(1024), 0, stream, osums, ob * kOrderClasses, status, cap);
        hipLaunchKernelGGL(k_order_write, dim3((unsigned)ob), dim3(256), 0, stream, ranges, nt, status, cap, osums, ob,
                           prefixed, order, order_bwd, items);
    }
    if (!radix) {
        // per-list sort from (kin, vin) into (kout, vout)
        hipLaunchKernelGGL(k_sort_short_lists, dim3((unsigned)nt), dim3(64), 0, stream, ranges, nt, status, cap, kin,
                           vin, kout, vout, long_list, reinterpret_cast<const uint32_t*>(vws + L.order_bwd));
        const int64_t lblocks = nt < 512 ? nt : 512;
        hipLaunchKernelGGL(k_sort_long_lists, dim3((unsigned)lblocks), dim3(256), 0, stream, ranges, long_list, status,
                           cap, kin, vin, kout, vout);
        *result_in_b = (kout == kb) ? 1 : 0;
    } else {
        *result_in_b = (kin == kb) ? 1 : 0;
    }
    return hipGetLastError();
}

}  // namespace linprim
