// Tile binning with a depth sort (the rasterizer front end of Sec. 4.4):
//   1. depth sort: stable LSD radix sort (4 x 8-bit digits) of the kept
//      Gaussians by the bits of their FP32 depth (positive floats order like
//      their bit patterns), values = frame-local Gaussian index; the first
//      pass also drops culled Gaussians (compaction).
//   2. exclusive scan of the tiles of each sorted Gaussian's footprint -> pair
//      offsets.
//   3. emit: every output pair (tile, Gaussian) is written by one lane
//      (load-balanced over pairs, not over Gaussians), staged in LDS and
//      stored coalesced; pairs come out in depth order.
//   4. tile sort: stable LSD radix sort of the pairs by tile id; stability
//      keeps the depth order inside each tile, so each tile list is ordered by
//      (depth bits, Gaussian index).
//   5. ranges: [begin, end) of every tile's list.
// Every stage is segmented by frame: a frame's elements never mix with
// another frame's, so a frame bins identically alone and in a batch.
// Sizes that depend on the data (kept Gaussians, pairs) stay on the device;
// the kernels that need them run persistent grids over work tiles.
#include "common.h"
#include "footprint.h"
#include "gload.h"

namespace sd7 {

// ---------------------------------------------------------------------------
// block-wide exclusive scan of one value per thread (256 threads)
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t block_excl_scan(uint32_t x, uint32_t* s_tmp, uint32_t& total)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    uint32_t v = x;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const uint32_t t = __shfl_up(v, off);
        if (lane >= off) v += t;
    }
    if (lane == 63) s_tmp[wave] = v;
    __syncthreads();
    uint32_t before = 0;
    total = 0;
#pragma unroll
    for (int w = 0; w < 4; ++w) {
        const uint32_t s = s_tmp[w];
        if (w < wave) before += s;
        total += s;
    }
    __syncthreads();
    return before + v - x;
}

// ---------------------------------------------------------------------------
// device-wide exclusive scan (reduce, spine, down-sweep); length given either
// on the host (len_dev == nullptr) or in device memory.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_scan_reduce(const uint32_t* __restrict__ in, uint32_t len_host,
                                                     const uint32_t* __restrict__ len_dev,
                                                     uint32_t* __restrict__ partials)
{
    __shared__ uint32_t s_tmp[4];
    const uint32_t len = len_dev ? *len_dev : len_host;
    const uint32_t ntiles = (len + kScanItems - 1) / kScanItems;
    for (uint32_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
        const uint32_t base = t * kScanItems + threadIdx.x * 16;
        uint32_t s = 0;
        if (base + 16 <= len) {
            const uint4* p = reinterpret_cast<const uint4*>(in + base);
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const uint4 q = p[k];
                s += q.x + q.y + q.z + q.w;
            }
        } else {
            for (uint32_t e = base; e < len && e < base + 16; ++e) s += in[e];
        }
        uint32_t total;
        block_excl_scan(s, s_tmp, total);
        if (threadIdx.x == 0) partials[t] = total;
    }
}

// One block: exclusive scan of the partials in place; the grand total goes to
// partials[ntiles] and, if requested, to *total_out.
__global__ __launch_bounds__(1024) void k_scan_spine(uint32_t* __restrict__ partials, uint32_t len_host,
                                                     const uint32_t* __restrict__ len_dev,
                                                     uint32_t* __restrict__ total_out)
{
    __shared__ uint32_t s_w[16];
    __shared__ uint32_t s_carry;
    const uint32_t len = len_dev ? *len_dev : len_host;
    const uint32_t ntiles = (len + kScanItems - 1) / kScanItems;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (threadIdx.x == 0) s_carry = 0;
    __syncthreads();
    for (uint32_t base = 0; base < ntiles; base += 1024) {
        const uint32_t e = base + threadIdx.x;
        const uint32_t x = e < ntiles ? partials[e] : 0;
        uint32_t v = x;
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const uint32_t t = __shfl_up(v, off);
            if (lane >= off) v += t;
        }
        if (lane == 63) s_w[wave] = v;
        __syncthreads();
        uint32_t before = s_carry, tot = s_carry;
        for (int w = 0; w < 16; ++w) {
            if (w < wave) before += s_w[w];
            tot += s_w[w];
        }
        if (e < ntiles) partials[e] = before + v - x;
        __syncthreads();
        if (threadIdx.x == 0) s_carry = tot;
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        partials[ntiles] = s_carry;
        if (total_out) *total_out = s_carry;
    }
}

// Down-sweep: each work tile's exclusive scan plus the tile's carry.  SUMS:
// the partials are the raw tile sums and each tile adds up those before it
// itself (no spine pass; for scans of at most kScanCarryTiles tiles), and the
// last tile writes the grand total to *total_out; otherwise the partials hold
// the spine's exclusive carries.
constexpr uint32_t kScanCarryTiles = 2048;

template <bool SUMS>
__global__ __launch_bounds__(256) void k_scan_down(const uint32_t* in, uint32_t* out, uint32_t len_host,
                                                   const uint32_t* __restrict__ len_dev,
                                                   const uint32_t* __restrict__ partials,
                                                   uint32_t* __restrict__ total_out)
{
    __shared__ uint32_t s_tmp[4];
    const uint32_t len = len_dev ? *len_dev : len_host;
    const uint32_t ntiles = (len + kScanItems - 1) / kScanItems;
    if (SUMS && ntiles == 0 && total_out && blockIdx.x == 0 && threadIdx.x == 0) *total_out = 0;
    for (uint32_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
        uint32_t carry;
        if (SUMS) {
            uint32_t c = 0;
            for (uint32_t i = threadIdx.x; i < t; i += 256) c += partials[i];
            uint32_t ctot;
            block_excl_scan(c, s_tmp, ctot);
            carry = ctot;
        } else {
            carry = partials[t];
        }
        const uint32_t base = t * kScanItems + threadIdx.x * 16;
        uint32_t v[16];
        const bool full = base + 16 <= len;
        if (full) {
            const uint4* p = reinterpret_cast<const uint4*>(in + base);
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const uint4 q = p[k];
                v[4 * k] = q.x; v[4 * k + 1] = q.y; v[4 * k + 2] = q.z; v[4 * k + 3] = q.w;
            }
        } else {
#pragma unroll
            for (int k = 0; k < 16; ++k) v[k] = (base + k < len) ? in[base + k] : 0;
        }
        uint32_t s = 0;
#pragma unroll
        for (int k = 0; k < 16; ++k) s += v[k];
        uint32_t total;
        uint32_t run = block_excl_scan(s, s_tmp, total) + carry;
        if (SUMS && t + 1 == ntiles && total_out && threadIdx.x == 0) *total_out = carry + total;
#pragma unroll
        for (int k = 0; k < 16; ++k) {
            const uint32_t x = v[k];
            v[k] = run;
            run += x;
        }
        if (full) {
            uint4* p = reinterpret_cast<uint4*>(out + base);
#pragma unroll
            for (int k = 0; k < 4; ++k) p[k] = make_uint4(v[4 * k], v[4 * k + 1], v[4 * k + 2], v[4 * k + 3]);
        } else {
#pragma unroll
            for (int k = 0; k < 16; ++k)
                if (base + k < len) out[base + k] = v[k];
        }
    }
}

// ---------------------------------------------------------------------------
// segmented LSD radix sort, one 8-bit digit per pass
// histogram layout: hist[256 * seg.wt0 + digit * seg.nwt + tile_in_seg]; an
// exclusive scan over the flat array then gives every (segment, digit, tile)
// its first output slot, minus the elements of earlier segments.
// ---------------------------------------------------------------------------
template <bool FIRST>
__global__ __launch_bounds__(256) void k_radix_hist(const uint32_t* __restrict__ keys,
                                                    const SortSeg* __restrict__ segs, int nseg,
                                                    const SortTotals* __restrict__ tot, int shift,
                                                    uint32_t* __restrict__ hist)
{
    __shared__ uint32_t h[256];
    const uint32_t nwt = tot->wt;
    for (uint32_t w = blockIdx.x; w < nwt; w += gridDim.x) {
        const int s = seg_of_tile(segs, nseg, w);
        const SortSeg sg = segs[s];
        const uint32_t k = w - sg.wt0;
        h[threadIdx.x] = 0;
        __syncthreads();
        const uint32_t begin = k * kSortItems;
        const uint32_t end = min(sg.len, begin + kSortItems);
        for (uint32_t e = begin + threadIdx.x; e < end; e += 256) {
            const uint32_t key = keys[sg.in_base + e];
            if (FIRST && key == kCulled) continue;
            atomicAdd(&h[(key >> shift) & 255u], 1u);
        }
        __syncthreads();
        hist[256u * sg.wt0 + threadIdx.x * sg.nwt + k] = h[threadIdx.x];
        __syncthreads();
    }
}

// Stable scatter.  Wave w of a work tile owns elements [w*512, (w+1)*512)
// of the tile and ranks them in kSortPerThread rounds of 64 (wave-level
// multisplit: eight ballots find the lanes that share a digit); the per-wave
// digit counts are then scanned across waves and over the digits.  The tile's
// elements are placed in digit order in LDS and written out from there, so
// each store covers whole runs of one digit rather than one element per run.
template <bool FIRST>
__global__ __launch_bounds__(256) void k_radix_scatter(const uint32_t* __restrict__ keys_in,
                                                       const uint32_t* __restrict__ vals_in,
                                                       uint32_t* __restrict__ keys_out,
                                                       uint32_t* __restrict__ vals_out,
                                                       const SortSeg* __restrict__ segs, int nseg,
                                                       const SortTotals* __restrict__ tot, int shift,
                                                       const uint32_t* __restrict__ hist)
{
    __shared__ uint32_t s_goff[256];
    __shared__ uint32_t s_wh[4][256];
    __shared__ uint32_t s_dst[256];  // first position of each digit in the tile (digit order)
    __shared__ uint32_t s_tmp[4];
    __shared__ uint32_t s_key[kSortItems], s_val[kSortItems];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const uint64_t lt = lanemask_lt();
    const uint32_t nwt = tot->wt;
    for (uint32_t w = blockIdx.x; w < nwt; w += gridDim.x) {
        const int s = seg_of_tile(segs, nseg, w);
        const SortSeg sg = segs[s];
        const uint32_t k = w - sg.wt0;
        s_goff[tid] = hist[256u * sg.wt0 + tid * sg.nwt + k] - sg.cnt_excl + sg.out_base;
        s_wh[0][tid] = 0; s_wh[1][tid] = 0; s_wh[2][tid] = 0; s_wh[3][tid] = 0;
        __syncthreads();
        const uint32_t wbase = k * kSortItems + wave * (kSortPerThread * 64);
        uint32_t key[kSortPerThread], val[kSortPerThread], rank[kSortPerThread];
        uint32_t okmask = 0;
#pragma unroll
        for (int r = 0; r < kSortPerThread; ++r) {
            const uint32_t e = wbase + r * 64 + lane;
            bool ok = e < sg.len;
            const uint32_t kk = ok ? keys_in[sg.in_base + e] : 0u;
            if (FIRST) ok = ok && kk != kCulled;
            const uint32_t vv = FIRST ? e : (ok ? vals_in[sg.in_base + e] : 0u);
            const uint32_t d = (kk >> shift) & 255u;
            uint64_t peers = __ballot(ok);
#pragma unroll
            for (int b = 0; b < 8; ++b) {
                const bool bit = (d >> b) & 1u;
                const uint64_t bb = __ballot(bit);
                peers &= bit ? bb : ~bb;
            }
            const uint32_t below = __popcll(peers & lt);
            uint32_t prev = 0;
            if (ok) prev = s_wh[wave][d];
            if (ok && below == 0) s_wh[wave][d] = prev + __popcll(peers);
            key[r] = kk;
            val[r] = vv;
            rank[r] = prev + below;
            okmask |= (ok ? 1u : 0u) << r;
        }
        __syncthreads();
        uint32_t run = 0;  // the tile's count of digit tid
#pragma unroll
        for (int w2 = 0; w2 < 4; ++w2) {
            const uint32_t t = s_wh[w2][tid];
            s_wh[w2][tid] = run;
            run += t;
        }
        // exclusive scan of the digit counts over the 256 digits
        {
            uint32_t v = run;
#pragma unroll
            for (int off = 1; off < 64; off <<= 1) {
                const uint32_t t = __shfl_up(v, off);
                if (lane >= off) v += t;
            }
            if (lane == 63) s_tmp[wave] = v;
            __syncthreads();
            uint32_t before = 0;
#pragma unroll
            for (int w2 = 0; w2 < 4; ++w2)
                if (w2 < wave) before += s_tmp[w2];
            s_dst[tid] = before + v - run;
        }
        __syncthreads();
#pragma unroll
        for (int r = 0; r < kSortPerThread; ++r) {
            if ((okmask >> r) & 1u) {
                const uint32_t d = (key[r] >> shift) & 255u;
                const uint32_t q = s_dst[d] + s_wh[wave][d] + rank[r];
                s_key[q] = key[r];
                s_val[q] = val[r];
            }
        }
        __syncthreads();
        const uint32_t ntile = s_tmp[0] + s_tmp[1] + s_tmp[2] + s_tmp[3];  // elements the tile keeps
        for (uint32_t q = tid; q < ntile; q += 256) {
            const uint32_t kk = s_key[q];
            const uint32_t d = (kk >> shift) & 255u;
            const uint32_t p = s_goff[d] + (q - s_dst[d]);
            keys_out[p] = kk;
            vals_out[p] = s_val[q];
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// depth sort of a small call: one launch per 8-bit digit
//
// For calls of few work tiles the sort's launches, not its bytes, set its
// time.  k_depth_hist counts, per frame, the kept keys of each value of each
// of the four digits in one read of the keys; a digit's first output slot in
// the frame is the sum of the counts of the digits below it.  Each pass then
// ranks its work tiles like k_radix_scatter, and a tile finds how many keys
// of each digit the frame's earlier tiles hold by looking back over their
// published counts (decoupled look-back): a tile publishes its own counts as
// soon as it has them, then adds up earlier tiles' counts, newest first,
// until it meets one that already holds the inclusive sum over all tiles
// before it, and publishes that sum for its own successors.  Tiles take
// their index from a counter in the order their blocks start, so a tile only
// ever waits on tiles whose blocks are already running and publish without
// waiting; each wait is still bounded (kLookbackSpins polls) and a wait that
// gives up flags the frame with SD7_FLAG_SORT_STALL.  Both sorts give the
// same order.
// ---------------------------------------------------------------------------
constexpr uint32_t kStatAgg = 1u << 30;    // status word: the tile's own digit count
constexpr uint32_t kStatIncl = 2u << 30;   // status word: inclusive count over the frame's tiles so far
constexpr uint32_t kStatCount = (1u << 30) - 1u;
constexpr uint32_t kLookbackSpins = 1u << 22;  // polls of an unpublished tile before a wait gives up
constexpr int kLookWindow = 16;                 // earlier tiles a look-back step reads at once

// Per frame, the kept keys of every value of every digit: dh[f][digit][256].
// The block that counts work tile w also zeroes the tile's status words of
// the four passes (stat + p * sw + 256 w), which the passes then publish in.
__global__ __launch_bounds__(256) void k_depth_hist(const uint32_t* __restrict__ keys,
                                                    const SortSeg* __restrict__ segs, int nseg,
                                                    const SortTotals* __restrict__ tot, uint32_t* __restrict__ dh,
                                                    uint32_t* __restrict__ stat, size_t sw)
{
    __shared__ uint32_t h[4][256];
    const uint32_t nwt = tot->wt;
    for (uint32_t w = blockIdx.x; w < nwt; w += gridDim.x) {
#pragma unroll
        for (int p = 0; p < 4; ++p) stat[p * sw + (size_t)w * 256 + threadIdx.x] = 0;
        const int s = seg_of_tile(segs, nseg, w);
        const SortSeg sg = segs[s];
        h[0][threadIdx.x] = 0; h[1][threadIdx.x] = 0; h[2][threadIdx.x] = 0; h[3][threadIdx.x] = 0;
        __syncthreads();
        const uint32_t begin = (w - sg.wt0) * kSortItems;
        const uint32_t end = min(sg.len, begin + kSortItems);
        for (uint32_t e0 = begin; e0 < end; e0 += 256) {  // uniform trip count
            const uint32_t e = e0 + threadIdx.x;
            const uint32_t key = e < end ? keys[sg.in_base + e] : kCulled;
            const bool ok = key != kCulled;
            if (ok) {
                atomicAdd(&h[0][key & 255u], 1u);
                atomicAdd(&h[1][(key >> 8) & 255u], 1u);
                atomicAdd(&h[2][(key >> 16) & 255u], 1u);
            }
            // the top digit takes few values: one add per value and wave
            const uint32_t top = key >> 24;
            uint64_t act = __ballot(ok);
            while (act) {
                const int first = __builtin_ctzll(act);
                const uint32_t v = __builtin_amdgcn_readlane(top, first);
                const uint64_t peers = __ballot(ok && top == v);
                if ((int)__lane_id() == first) atomicAdd(&h[3][v], (uint32_t)__popcll(peers));
                act &= ~peers;
            }
        }
        __syncthreads();
        uint32_t* out = dh + (size_t)s * 1024;
#pragma unroll
        for (int d = 0; d < 4; ++d) {
            const uint32_t v = h[d][threadIdx.x];
            if (v) atomicAdd(&out[d * 256 + threadIdx.x], v);
        }
        __syncthreads();
    }
}

// One pass of the small call's depth sort over digit `digit` (bits 8 * digit
// ..).  FIRST: the keys of every Gaussian, culled ones dropped, values =
// frame-local index; KEYS_OUT false: only the values are written (the last
// pass).  One work tile per block; stat holds 256 status words per work tile
// of this pass and tile_ctr the pass's tile counter, both zero at the start.
template <bool FIRST, bool KEYS_OUT>
__global__ __launch_bounds__(256) void k_depth_pass(const uint32_t* __restrict__ keys_in,
                                                    const uint32_t* __restrict__ vals_in,
                                                    uint32_t* __restrict__ keys_out,
                                                    uint32_t* __restrict__ vals_out,
                                                    const SortSeg* __restrict__ segs, int nseg,
                                                    const SortTotals* __restrict__ tot, int digit,
                                                    const uint32_t* __restrict__ dh, uint32_t* stat,
                                                    uint32_t* tile_ctr, uint32_t* __restrict__ counts)
{
    __shared__ uint32_t s_goff[256];
    __shared__ uint32_t s_wh[4][256];
    __shared__ uint32_t s_dst[256];  // first position of each digit in the tile (digit order)
    __shared__ uint32_t s_tmp[4], s_base[4];
    __shared__ uint32_t s_key[kSortItems], s_val[kSortItems];
    __shared__ uint32_t s_w;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int shift = 8 * digit;
    if (tid == 0) s_w = atomicAdd(tile_ctr, 1u);
    __syncthreads();
    const uint32_t w = s_w;
    if (w >= tot->wt) return;  // uniform over the block
    const int s = seg_of_tile(segs, nseg, w);
    const SortSeg sg = segs[s];
    const uint32_t k = w - sg.wt0;
    s_wh[0][tid] = 0; s_wh[1][tid] = 0; s_wh[2][tid] = 0; s_wh[3][tid] = 0;
    // first output slot of digit tid in the frame: exclusive scan of the
    // frame's digit counts
    const uint32_t dcount = dh[(size_t)s * 1024 + digit * 256 + tid];
    {
        uint32_t v = dcount;
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const uint32_t t = __shfl_up(v, off);
            if (lane >= off) v += t;
        }
        if (lane == 63) s_base[wave] = v;
        __syncthreads();
        uint32_t before = 0;
#pragma unroll
        for (int w2 = 0; w2 < 4; ++w2)
            if (w2 < wave) before += s_base[w2];
        s_goff[tid] = sg.out_base + before + v - dcount;
    }
    const uint64_t lt = lanemask_lt();
    const uint32_t wbase = k * kSortItems + wave * (kSortPerThread * 64);
    uint32_t key[kSortPerThread], val[kSortPerThread], rank[kSortPerThread];
    uint32_t okmask = 0;
#pragma unroll
    for (int r = 0; r < kSortPerThread; ++r) {
        const uint32_t e = wbase + r * 64 + lane;
        bool ok = e < sg.len;
        const uint32_t kk = ok ? keys_in[sg.in_base + e] : 0u;
        if (FIRST) ok = ok && kk != kCulled;
        const uint32_t vv = FIRST ? e : (ok ? vals_in[sg.in_base + e] : 0u);
        const uint32_t d = (kk >> shift) & 255u;
        uint64_t peers = __ballot(ok);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            const bool bit = (d >> b) & 1u;
            const uint64_t bb = __ballot(bit);
            peers &= bit ? bb : ~bb;
        }
        const uint32_t below = __popcll(peers & lt);
        uint32_t prev = 0;
        if (ok) prev = s_wh[wave][d];
        if (ok && below == 0) s_wh[wave][d] = prev + __popcll(peers);
        key[r] = kk;
        val[r] = vv;
        rank[r] = prev + below;
        okmask |= (ok ? 1u : 0u) << r;
    }
    __syncthreads();
    uint32_t run = 0;  // the tile's count of digit tid
#pragma unroll
    for (int w2 = 0; w2 < 4; ++w2) {
        const uint32_t t = s_wh[w2][tid];
        s_wh[w2][tid] = run;
        run += t;
    }
    // publish the tile's count of digit tid, then look back
    uint32_t* const my = stat + (size_t)w * 256 + tid;
    __hip_atomic_store(my, (k == 0 ? kStatIncl : kStatAgg) | run, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    uint32_t excl = 0;
    if (k > 0) {
        // examine the earlier tiles kLookWindow at a time (independent loads),
        // newest first, up to the first one that has not published yet
        bool stalled = false;
        uint32_t j = w, polls = 0;  // tiles below j are still to be added
        for (;;) {
            uint32_t v[kLookWindow];
#pragma unroll
            for (int q = 0; q < kLookWindow; ++q) {
                const uint32_t jj = j - 1u - (uint32_t)q;
                // before the frame's first tile: an inclusive count of zero
                v[q] = (jj >= sg.wt0 && jj < j)
                           ? __hip_atomic_load(stat + (size_t)jj * 256 + tid, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)
                           : kStatIncl;
            }
            uint32_t used = 0;
            bool done = false;
#pragma unroll
            for (int q = 0; q < kLookWindow; ++q) {
                if (!done && used == (uint32_t)q && (v[q] & (kStatAgg | kStatIncl))) {
                    excl += v[q] & kStatCount;
                    used = q + 1;
                    done = (v[q] & kStatIncl) != 0;
                }
            }
            if (done) break;
            j -= used;
            if (used == 0) {
                if (++polls > kLookbackSpins) {
                    stalled = true;
                    break;
                }
                __builtin_amdgcn_s_sleep(1);
            }
        }
        __hip_atomic_store(my, kStatIncl | (excl + run), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (stalled) atomicOr(&counts[s * SD7_CNT_WORDS + SD7_CNT_FLAGS], SD7_FLAG_SORT_STALL);
    }
    s_goff[tid] += excl;
    // exclusive scan of the tile's digit counts over the 256 digits
    {
        uint32_t v = run;
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const uint32_t t = __shfl_up(v, off);
            if (lane >= off) v += t;
        }
        if (lane == 63) s_tmp[wave] = v;
        __syncthreads();
        uint32_t before = 0;
#pragma unroll
        for (int w2 = 0; w2 < 4; ++w2)
            if (w2 < wave) before += s_tmp[w2];
        s_dst[tid] = before + v - run;
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < kSortPerThread; ++r) {
        if ((okmask >> r) & 1u) {
            const uint32_t d = (key[r] >> shift) & 255u;
            const uint32_t q = s_dst[d] + s_wh[wave][d] + rank[r];
            s_key[q] = key[r];
            s_val[q] = val[r];
        }
    }
    __syncthreads();
    const uint32_t ntile = s_tmp[0] + s_tmp[1] + s_tmp[2] + s_tmp[3];  // elements the tile keeps
    for (uint32_t q = tid; q < ntile; q += 256) {
        const uint32_t kk = s_key[q];
        const uint32_t d = (kk >> shift) & 255u;
        const uint32_t p = s_goff[d] + (q - s_dst[d]);
        if (KEYS_OUT) keys_out[p] = kk;
        vals_out[p] = s_val[q];
    }
}

// ---------------------------------------------------------------------------
// set-up, gather, emit, ranges
// ---------------------------------------------------------------------------
__global__ void k_fill_u32(uint32_t* __restrict__ p, size_t count, uint32_t value)
{
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (size_t)gridDim.x * blockDim.x)
        p[i] = value;
}

__global__ void k_copy_u32(uint32_t* __restrict__ dst, const uint32_t* __restrict__ src, uint32_t count)
{
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < count; i += gridDim.x * blockDim.x) dst[i] = src[i];
}

// Segments of the depth sort.  segs_all: every Gaussian (the compacting first
// pass); segs_kept: the kept ones.  One wave, lane f = frame f (at most 64
// frames); offsets are wave prefix sums.
__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t v, uint32_t lane)
{
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const uint32_t t = __shfl_up(v, off);
        if (lane >= (uint32_t)off) v += t;
    }
    return v;
}

// Depth order of calls whose frames hold at most kSmallSortItems Gaussians
// each: one block per frame sorts (depth key, index) pairs in LDS with a
// bitonic network and writes the kept Gaussians' indices in that order (the
// order the radix passes give: depth, then index; culled keys, all ones, sort
// last).  One launch in place of the setup, the digit count and four digit
// passes, which a call of a thousand Gaussians spends most of its time
// launching.
constexpr uint32_t kSmallSortItems = 2048;
constexpr uint32_t kSmallSortThreads = kSmallSortItems / 2;  // one compare-exchange per thread and step

__global__ __launch_bounds__(kSmallSortThreads) void k_depth_small(const FrameDev* __restrict__ tab,
                                                                   const uint32_t* __restrict__ counts,
                                                                   const uint32_t* __restrict__ dkey,
                                                                   uint32_t* __restrict__ order)
{
    __shared__ uint64_t s_k[kSmallSortItems];
    const FrameDev& F = tab[blockIdx.x];
    const uint32_t n = F.n, tid = threadIdx.x;
    uint32_t m = 64;  // a power of two >= n (all threads take part in every step)
    while (m < n) m <<= 1;
    for (uint32_t i = tid; i < m; i += kSmallSortThreads)
        s_k[i] = i < n ? (uint64_t)dkey[F.g0 + i] << 32 | i : ~0ull;
    __syncthreads();
    for (uint32_t k = 2; k <= m; k <<= 1) {
        for (uint32_t j = k >> 1; j > 0; j >>= 1) {
            const uint32_t i = 2 * tid - (tid & (j - 1));  // the pair (i, i + j), i's bit j clear
            if (i + j < m) {
                const uint64_t a = s_k[i], b = s_k[i + j];
                if ((a > b) == ((i & k) == 0)) {  // ascending where bit k of i is clear
                    s_k[i] = b;
                    s_k[i + j] = a;
                }
            }
            __syncthreads();
        }
    }
    const uint32_t kept = counts[blockIdx.x * SD7_CNT_WORDS + SD7_CNT_KEPT];
    for (uint32_t i = tid; i < kept; i += kSmallSortThreads) order[F.g0 + i] = (uint32_t)s_k[i];
}

// Also zeroes `clear` (clear_words words: the small call's digit counts and
// tile counters) with all 256 lanes; the first wave sets up the segments.
__global__ __launch_bounds__(256) void k_setup_depth(const FrameDev* __restrict__ tab, int nf,
                                                     const uint32_t* __restrict__ counts,
                                                     SortSeg* __restrict__ segs_all, SortTotals* __restrict__ tot_all,
                                                     SortSeg* __restrict__ segs_kept, SortTotals* __restrict__ tot_kept,
                                                     uint32_t* __restrict__ clear, uint32_t clear_words)
{
    for (uint32_t i = threadIdx.x; i < clear_words; i += blockDim.x) clear[i] = 0;
    if (threadIdx.x >= 64) return;
    const uint32_t lane = threadIdx.x;
    const bool live = (int)lane < nf;
    const uint32_t n = live ? tab[lane].n : 0u, g0 = live ? tab[lane].g0 : 0u;
    const uint32_t kept = live ? counts[lane * SD7_CNT_WORDS + SD7_CNT_KEPT] : 0u;
    const uint32_t nwa = (n + kSortItems - 1) / kSortItems, nwk = (kept + kSortItems - 1) / kSortItems;
    const uint32_t wa = wave_incl_scan(nwa, lane), wk = wave_incl_scan(nwk, lane);
    const uint32_t ex = wave_incl_scan(kept, lane);
    if (live) {
        SortSeg a;
        a.in_base = g0; a.out_base = g0; a.len = n; a.wt0 = wa - nwa;
        a.nwt = nwa; a.cnt_excl = ex - kept; a.pad[0] = a.pad[1] = 0;
        SortSeg b = a;
        b.len = kept; b.wt0 = wk - nwk; b.nwt = nwk;
        segs_all[lane] = a;
        segs_kept[lane] = b;
    }
    if (lane == 63) {
        tot_all->wt = wa; tot_all->hist_len = 256u * wa;
        tot_kept->wt = wk; tot_kept->hist_len = 256u * wk;
    }
}

// The counting binner's copy of a footprint.  A box of at most kMaskSide x
// kMaskSide tiles carries kMaskFlag in x and its covered tiles as a bit mask
// in z (rows 0..3) and w (rows 4..7), bit 8 * row + column; a larger box is
// the footprint itself (row trims in z and w).  x = x0 | y0 << 16 and
// y = x1 | y1 << 16 otherwise, as in the footprint (x0 < 1024, so bit 15 of
// x is free for the flag).
constexpr uint32_t kMaskSide = 8;
constexpr uint32_t kMaskFlag = 0x8000u;

__device__ __forceinline__ uint4 bin_box(uint4 f)
{
    const Footprint fp(f);
    if (fp.w() > kMaskSide || fp.h() > kMaskSide) return f;
    uint64_t m = 0;
    for (uint32_t r = 0; r < fp.h(); ++r) {
        int a, b;
        fp.row(r, a, b);
        if (a < b) m |= (((1ull << (b - a)) - 1ull) << (a - (int)fp.x0)) << (kMaskSide * r);
    }
    return make_uint4(f.x | kMaskFlag, f.y, (uint32_t)m, (uint32_t)(m >> 32));
}

// Tile columns [a, b) of row r (0 <= r < h) of a binner box; empty when a >= b.
__device__ __forceinline__ void bin_box_row(uint4 bb, uint32_t r, int& a, int& b)
{
    if (!(bb.x & kMaskFlag)) {
        Footprint(bb).row(r, a, b);
        return;
    }
    const int x0 = (int)(bb.x & 0x7FFFu);
    const uint32_t bits = ((r < 4 ? bb.z : bb.w) >> (8 * (r & 3u))) & 0xFFu;
    a = x0 + (int)__builtin_ctz(bits | 0x100u);
    b = x0 + 32 - (int)__builtin_clz(bits | 1u);
    if (bits == 0) b = a;
}

// Tile groups (kGroup x kGroup tiles) that the bounding box of a footprint
// meets, as bytes gx0 | (gx1 - gx0) << 8 | gy0 << 16 | (gy1 - gy0) << 24 with
// inclusive ends.  An empty box packs to all ones, which meets no group of a
// frame of at most 255 * kGroup tiles per side.
__device__ __forceinline__ uint32_t group_span(uint4 r)
{
    const uint32_t x0 = r.x & 0xFFFFu, y0 = r.x >> 16, x1 = r.y & 0xFFFFu, y1 = r.y >> 16;
    if (x0 >= x1 || y0 >= y1) return 0xFFFFFFFFu;
    const uint32_t gx0 = x0 / kGroup, gx1 = (x1 - 1) / kGroup;
    const uint32_t gy0 = y0 / kGroup, gy1 = (y1 - 1) / kGroup;
    return gx0 | (gx1 - gx0) << 8 | gy0 << 16 | (gy1 - gy0) << 24;
}

// Whether group (gx, gy) lies in a packed group span.
__device__ __forceinline__ bool span_meets(uint32_t d, uint32_t gx, uint32_t gy)
{
    return (gx - (d & 0xFFu) <= ((d >> 8) & 0xFFu)) & (gy - ((d >> 16) & 0xFFu) <= (d >> 24));
}

// Tiles of each Gaussian's footprint in depth order (0 past the kept ones).
__global__ __launch_bounds__(kBlock) void k_gather_ntiles(const FrameDev* __restrict__ tab, BlockMap bm,
                                                          const uint32_t* __restrict__ counts,
                                                          const uint32_t* __restrict__ order,
                                                          const uint4* __restrict__ rect,
                                                          uint32_t* __restrict__ ntiles)
{
    const int f = frame_of_block(bm, blockIdx.x);
    const FrameDev& F = tab[f];
    const uint32_t j = (blockIdx.x - bm.start[f]) * kBlock + threadIdx.x;
    if (j >= F.n) return;
    const uint32_t kept = counts[f * SD7_CNT_WORDS + SD7_CNT_KEPT];
    ntiles[F.g0 + j] = j < kept ? Footprint(rect[F.g0 + order[F.g0 + j]]).tiles() : 0u;
}

// The binner boxes and group spans of the kept footprints in depth order.
__global__ __launch_bounds__(kBlock) void k_gather_boxes(const FrameDev* __restrict__ tab, BlockMap bm,
                                                         const uint32_t* __restrict__ counts,
                                                         const uint32_t* __restrict__ order,
                                                         const uint4* __restrict__ rect,
                                                         uint4* __restrict__ srect,
                                                         uint32_t* __restrict__ sspan)
{
    const int f = frame_of_block(bm, blockIdx.x);
    const FrameDev& F = tab[f];
    const uint32_t j = (blockIdx.x - bm.start[f]) * kBlock + threadIdx.x;
    if (j >= counts[f * SD7_CNT_WORDS + SD7_CNT_KEPT]) return;
    const uint4 r = rect[F.g0 + order[F.g0 + j]];
    srect[F.g0 + j] = bin_box(r);
    sspan[F.g0 + j] = group_span(r);
}

// Per-frame pair counts, arena slots (each frame's share rounded up to a whole
// number of sort work tiles) and the tile-sort segments.  The pair counts come
// from an exclusive scan over all frames of the tiles per sorted Gaussian
// (by_tiles false) or of the pairs per tile (by_tiles true), each frame's
// elements contiguous.  One wave, lane f = frame f: the frames' pair counts
// are read in parallel; the arena is then handed out in frame order (a frame
// that does not fit gets none, and later frames may still fit), a walk over
// values already in registers.
// The work of one wave (lane = threadIdx.x % 64 < 64 frames); returns the
// lane's frame's pair count and first arena slot (0 for lanes past nf).
__device__ __forceinline__ uint2 setup_pairs_wave(const FrameDev* __restrict__ tab, int nf, uint32_t len_total,
                                                  bool by_tiles, const uint32_t* __restrict__ toff,
                                                  uint32_t total, uint32_t capacity,
                                                  uint32_t* __restrict__ counts, SortSeg* __restrict__ segs,
                                                  SortTotals* __restrict__ tot, uint32_t lane)
{
    const bool live = (int)lane < nf;
    uint32_t P = 0, lo = 0;
    if (live) {
        const FrameDev& F = tab[lane];
        const uint32_t e0 = by_tiles ? F.t0 : F.g0, ne = by_tiles ? F.tiles_x * F.tiles_y : F.n;
        lo = e0 < len_total ? toff[e0] : total;
        const uint32_t hi = (e0 + ne) < len_total ? toff[e0 + ne] : total;
        P = hi - lo;
    }
    uint32_t base = 0, wt = 0, excl = 0;
    uint32_t my_base = 0, my_wt = 0, my_excl = 0, my_len = 0;
    bool my_ov = false;
    for (int f = 0; f < nf; ++f) {
        const uint32_t Pf = __builtin_amdgcn_readlane(P, f);
        const bool ov = (uint64_t)base + Pf > capacity;
        const uint32_t len = ov ? 0u : Pf;
        const uint32_t nwt = (len + kSortItems - 1) / kSortItems;
        if (lane == (uint32_t)f) {
            my_base = base; my_wt = wt; my_excl = excl; my_len = len; my_ov = ov;
        }
        wt += nwt;
        excl += len;
        base += nwt * kSortItems;
    }
    if (live) {
        uint32_t* c = counts + lane * SD7_CNT_WORDS;
        // binning may be re-run with a larger arena: the flag is recomputed
        const uint32_t fl = c[SD7_CNT_FLAGS] & ~SD7_FLAG_PAIR_OVERFLOW;
        c[SD7_CNT_FLAGS] = my_ov ? (fl | SD7_FLAG_PAIR_OVERFLOW) : fl;
        c[SD7_CNT_PAIRS] = my_len;
        c[SD7_CNT_NEEDED] = P;
        c[SD7_CNT_PAIR_BASE] = my_base;
        c[5] = lo;  // scan value at the frame's first element
        SortSeg sg;
        sg.in_base = my_base; sg.out_base = my_base; sg.len = my_len; sg.wt0 = my_wt;
        sg.nwt = (my_len + kSortItems - 1) / kSortItems; sg.cnt_excl = my_excl; sg.pad[0] = sg.pad[1] = 0;
        segs[lane] = sg;
    }
    if (lane == 0) {
        tot->wt = wt;
        tot->hist_len = 256u * wt;
    }
    return make_uint2(my_len, my_base);
}

__global__ __launch_bounds__(64) void k_setup_pairs(const FrameDev* __restrict__ tab, int nf, uint32_t len_total,
                                                    bool by_tiles, const uint32_t* __restrict__ toff,
                                                    const uint32_t* __restrict__ toff_total, uint32_t capacity,
                                                    uint32_t* __restrict__ counts, SortSeg* __restrict__ segs,
                                                    SortTotals* __restrict__ tot)
{
    setup_pairs_wave(tab, nf, len_total, by_tiles, toff, *toff_total, capacity, counts, segs, tot, threadIdx.x);
}

// Tile id of the l-th tile of a footprint (row by row, left to right);
// l < tiles().
__device__ __forceinline__ uint32_t footprint_tile(const Footprint& fp, uint32_t l, uint32_t tiles_x)
{
    const uint32_t h = fp.h(), m = fp.first_bottom_row(), w = fp.w();
    int a, b;
    for (uint32_t r = 0; r < 4 && r < h; ++r) {
        const uint32_t n = fp.row_tiles(r);
        if (l < n) {
            fp.row(r, a, b);
            return (fp.y0 + r) * tiles_x + (uint32_t)a + l;
        }
        l -= n;
    }
    if (m > 4) {  // whole rows 4 .. m-1
        const uint32_t mid = (m - 4) * w;
        if (l < mid) return (fp.y0 + 4 + l / w) * tiles_x + fp.x0 + l % w;
        l -= mid;
    }
    uint32_t r = m;
    for (; r + 1 < h; ++r) {
        const uint32_t n = fp.row_tiles(r);
        if (l < n) break;
        l -= n;
    }
    fp.row(r, a, b);
    return (fp.y0 + r) * tiles_x + (uint32_t)a + l;
}

// Load-balanced emission: work tile w covers pairs [k*4096, (k+1)*4096) of
// one frame; each lane finds the Gaussian of its first pair by binary search
// over the pair offsets and walks forward.
__global__ __launch_bounds__(256) void k_emit(const FrameDev* __restrict__ tab, const uint32_t* __restrict__ counts,
                                              const uint32_t* __restrict__ order, const uint4* __restrict__ rect,
                                              const uint32_t* __restrict__ toff,
                                              const SortSeg* __restrict__ segs, int nseg,
                                              const SortTotals* __restrict__ tot,
                                              uint32_t* __restrict__ pair_tile, uint32_t* __restrict__ pair_g)
{
    __shared__ uint32_t s_t[kSortItems];
    __shared__ uint32_t s_g[kSortItems];
    const uint32_t nwt = tot->wt;
    for (uint32_t w = blockIdx.x; w < nwt; w += gridDim.x) {
        const int f = seg_of_tile(segs, nseg, w);
        const SortSeg sg = segs[f];
        const FrameDev& F = tab[f];
        const uint32_t kept = counts[f * SD7_CNT_WORDS + SD7_CNT_KEPT];
        const uint32_t lo = counts[f * SD7_CNT_WORDS + 5];
        const uint32_t k = w - sg.wt0;
        const uint32_t t_begin = k * kSortItems;
        const uint32_t cnt = min((uint32_t)kSortItems, sg.len - t_begin);
        const uint32_t o0 = t_begin + threadIdx.x * kSortPerThread;
        const uint32_t* tf = toff + F.g0;
        const uint32_t* of = order + F.g0;
        if (o0 < sg.len) {
            // largest j with tf[j] - lo <= o0
            uint32_t a = 0, b = kept - 1;
            while (a < b) {
                const uint32_t mid = (a + b + 1) >> 1;
                if (tf[mid] - lo <= o0) a = mid; else b = mid - 1;
            }
            uint32_t j = a;
            uint32_t start = tf[j] - lo;
            uint32_t next = (j + 1 < kept) ? tf[j + 1] - lo : sg.len;
            uint4 rc = rect[F.g0 + of[j]];
            uint32_t g = of[j];
#pragma unroll 1
            for (int r = 0; r < kSortPerThread; ++r) {
                const uint32_t o = o0 + r;
                if (o >= sg.len) break;
                while (o >= next) {
                    ++j;
                    start = next;
                    next = (j + 1 < kept) ? tf[j + 1] - lo : sg.len;
                    g = of[j];
                    rc = rect[F.g0 + g];
                }
                s_t[threadIdx.x * kSortPerThread + r] = footprint_tile(Footprint(rc), o - start, F.tiles_x);
                s_g[threadIdx.x * kSortPerThread + r] = g;
            }
        }
        __syncthreads();
        for (uint32_t e = threadIdx.x; e < cnt; e += 256) {
            pair_tile[sg.out_base + t_begin + e] = s_t[e];
            pair_g[sg.out_base + t_begin + e] = s_g[e];
        }
        __syncthreads();
    }
}

__global__ __launch_bounds__(256) void k_ranges(const FrameDev* __restrict__ tab, const uint32_t* __restrict__ pair_tile,
                                                const SortSeg* __restrict__ segs, int nseg,
                                                const SortTotals* __restrict__ tot, uint2* __restrict__ ranges)
{
    const uint32_t nwt = tot->wt;
    for (uint32_t w = blockIdx.x; w < nwt; w += gridDim.x) {
        const int f = seg_of_tile(segs, nseg, w);
        const SortSeg sg = segs[f];
        const uint32_t t0 = tab[f].t0;
        const uint32_t ntile = tab[f].tiles_x * tab[f].tiles_y;
        const uint32_t k = w - sg.wt0;
        const uint32_t end = min(sg.len, (k + 1) * kSortItems);
        for (uint32_t e = k * kSortItems + threadIdx.x; e < end; e += 256) {
            const uint32_t i = sg.in_base + e;
            const uint32_t t = pair_tile[i];
            if (t >= ntile) continue;  // never true for well-formed pairs
            if (e == 0 || pair_tile[i - 1] != t) ranges[t0 + t].x = i;
            if (e + 1 == sg.len || pair_tile[i + 1] != t) ranges[t0 + t].y = i + 1;
        }
    }
}

// ---------------------------------------------------------------------------
// counting binner: tile lists straight from the depth-sorted tile boxes
//
// The kept Gaussians of a frame, in depth order, are cut into nch chunks.
// k_tile_count writes how many of each chunk's boxes cover each tile into a
// [chunk][tile] matrix; a per-tile exclusive prefix over the chunks and a
// scan of the tile totals give every (chunk, tile) run its first arena slot,
// so the runs of one tile follow each other in depth order.  k_group_place
// then runs one wave per (chunk, group of 8 x 8 tiles), one lane per tile: it
// scans the 4-byte group spans of the chunk's boxes in depth order, fetches
// the boxes that meet the group, visits them one at a time, and every lane
// whose tile the box covers appends the Gaussian to its run (staged in LDS,
// written out as runs).  Each tile list thus comes out in (depth, index)
// order without a sort over pairs, and every wave writes only its own 64 runs.
// ---------------------------------------------------------------------------

__device__ __forceinline__ uint32_t frame_kept(const uint32_t* counts, int f)
{
    return counts[f * SD7_CNT_WORDS + SD7_CNT_KEPT];
}

// First depth-sorted Gaussian of chunk c when kept Gaussians are cut into
// nch chunks of equal size (multiples of 64, the last one shorter).
__device__ __forceinline__ uint32_t chunk_begin(uint32_t kept, uint32_t nch, uint32_t c)
{
    const uint32_t len = ((kept + nch - 1) / nch + 63) & ~63u;
    return min(kept, c * len);
}

// Entries of one placement pipeline stage, in units of 64 (one per lane).
constexpr int kBinAhead = 1;

// Appends a counting-binner lane stages in LDS before the wave writes them
// out, kStageDepth per tile.  A flush writes kStageTiles tiles per store, one
// lane per staged append; rows of the stage are kStagePitch words apart, which
// puts the 32 lanes of a half-wave in 32 different banks when a flush reads.
constexpr uint32_t kStageDepth = 16;
constexpr uint32_t kStageTiles = 64 / kStageDepth;
constexpr uint32_t kStagePitch = 64 + 32 / kStageDepth;
static_assert(kStageDepth * kStageTiles == 64 && kStageDepth <= 32, "a flush store covers whole tiles");
constexpr uint32_t kFlushAhead = 2;  // flush stores whose stage reads are issued together

// s_waitcnt operand that waits for the LDS/scalar-memory counter only
// (lgkmcnt 0; vmcnt and expcnt at their maxima).
constexpr int kWaitLgkm0 = 0xC07F;


// One block (256 lanes) per (frame, chunk) writes the chunk's row of the
// count matrix.  Per-row difference array over the frame's tiles in LDS: a
// footprint whose row y spans tiles [a, b) adds +1 at (a, y) and -1 at (b, y).
__global__ __launch_bounds__(256) void k_tile_count(const FrameDev* __restrict__ tab, BlockMap cm,
                                                    const uint32_t* __restrict__ counts,
                                                    const uint4* __restrict__ srect,
                                                    uint32_t* __restrict__ cnt)
{
    extern __shared__ uint32_t s_d[];
    const int f = frame_of_block(cm, blockIdx.x);
    const FrameDev& F = tab[f];
    const uint32_t c = blockIdx.x - cm.start[f];
    const uint32_t tx = F.tiles_x, T = F.tiles_x * F.tiles_y;
    for (uint32_t i = threadIdx.x; i < T; i += 256) s_d[i] = 0;
    __syncthreads();
    const uint32_t kept = frame_kept(counts, f);
    const uint32_t j0 = chunk_begin(kept, F.nch, c), j1 = chunk_begin(kept, F.nch, c + 1);
    for (uint32_t j = j0 + threadIdx.x; j < j1; j += 256) {
        const uint4 bb = srect[F.g0 + j];
        const Footprint fp(make_uint4(bb.x & ~kMaskFlag, bb.y, bb.z, bb.w));
        if (!(bb.x & kMaskFlag) && !fp.trimmed()) {
            for (uint32_t y = fp.y0; y < fp.y1; ++y) {
                atomicAdd(&s_d[y * tx + fp.x0], 1u);
                if (fp.x1 < tx) atomicSub(&s_d[y * tx + fp.x1], 1u);
            }
            continue;
        }
        for (uint32_t r = 0; r < fp.h(); ++r) {
            int a, b;
            bin_box_row(bb, r, a, b);
            if (a >= b) continue;
            const uint32_t y = fp.y0 + r;
            atomicAdd(&s_d[y * tx + a], 1u);
            if ((uint32_t)b < tx) atomicSub(&s_d[y * tx + b], 1u);
        }
    }
    __syncthreads();
    for (uint32_t y = threadIdx.x; y < F.tiles_y; y += 256) {
        uint32_t run = 0;
        for (uint32_t x = 0; x < tx; ++x) {
            run += s_d[y * tx + x];
            s_d[y * tx + x] = run;
        }
    }
    __syncthreads();
    uint32_t* row = cnt + F.m0 + (size_t)c * T;
    for (uint32_t t = threadIdx.x; t < T; t += 256) row[t] = s_d[t];
}

// One wave per (frame, chunk, group of kGroup x kGroup tiles), one lane per
// tile of the group: appends the chunk's Gaussians, in depth order, to the
// runs of the group's tiles, starting at the slots the scans gave.  Logical
// block b of a frame is chunk b / groups, group b % groups, and logical
// blocks are laid out contiguously per XCD, so the groups of one chunk run
// side by side on one XCD and share its group spans in that XCD's L2.
//
// The wave reads the chunk's 4-byte group spans, a set of kBinAhead * 64 at a
// time; only the lanes whose entry meets the group fetch its binner box and
// Gaussian index.  Three sets are in flight: the spans of the next one or
// two, the boxes of the current one, and the set being visited.  Each lane
// stages its appends in LDS (kStageDepth per tile); when one lane's stage is
// full, and at the end, the wave writes the staged runs out with all its
// lanes, kStageTiles tiles per store (the last flush, when no tile holds
// more than half a stage, one stage row per store), so the arena receives
// runs rather than scattered 4-byte stores.
__global__ __launch_bounds__(64) void k_group_place(const FrameDev* __restrict__ tab, BlockMap cm,
                                                    const uint32_t* __restrict__ counts,
                                                    const uint32_t* __restrict__ order,
                                                    const uint4* __restrict__ srect,
                                                    const uint32_t* __restrict__ sspan,
                                                    const uint32_t* __restrict__ cnt_pre,
                                                    const uint32_t* __restrict__ tstart,
                                                    uint32_t* __restrict__ pair_g)
{
    constexpr uint32_t kSet = kBinAhead * 64;
    const uint32_t lb = xcd_contiguous(blockIdx.x, gridDim.x);
    const int f = frame_of_block(cm, lb);
    const uint32_t b = lb - cm.start[f];
    const FrameDev& F = tab[f];
    const uint32_t tx = F.tiles_x, ty = F.tiles_y, T = tx * ty;
    const uint32_t gxn = (tx + kGroup - 1) / kGroup;
    const uint32_t ngr = gxn * ((ty + kGroup - 1) / kGroup);
    const uint32_t c = b / ngr, gr = b - c * ngr;
    const uint32_t gx = gr % gxn, gy = gr / gxn;
    const uint32_t lane = threadIdx.x;
    const uint32_t lx = gx * kGroup + (lane % kGroup), ly = gy * kGroup + (lane / kGroup);
    const bool valid = lx < tx && ly < ty;
    const uint32_t t = ly * tx + lx;
    const uint32_t* cf = counts + f * SD7_CNT_WORDS;
    const uint32_t kept = cf[SD7_CNT_KEPT];
    const uint32_t j0 = chunk_begin(kept, F.nch, c), j1 = chunk_begin(kept, F.nch, c + 1);
    if (cf[SD7_CNT_PAIRS] == 0 || j0 >= j1) return;  // uniform over the wave
    __shared__ uint32_t s_stage[(kStageDepth + 1) * kStagePitch];  // [depth][lane], and a spare row
    // LDS pointers (address space 3), so the stage is written with LDS stores
    using lds_u32 = __attribute__((address_space(3))) uint32_t;
    lds_u32* const s_lane = (lds_u32*)(s_stage + lane);  // the lane's column
    lds_u32* const s_end = s_lane + kStageDepth * kStagePitch;
    lds_u32* sp = s_lane;  // next free row of the lane's column
    uint32_t slot = 0;      // arena slot of the lane's first staged append
    {
        const uint32_t* ts = tstart + F.t0;
        if (valid) slot = cf[SD7_CNT_PAIR_BASE] + (ts[t] - ts[0]) + cnt_pre[F.m0 + (size_t)c * T + t];
    }
    const uint4* rf = srect + F.g0;
    const uint32_t* of = order + F.g0;
    const uint32_t* sf = sspan + F.g0;
    // spans of entries jb + k * 64 + lane, loaded in bounds (from j1 - 1 past the chunk)
    auto load_spans = [&](uint32_t (&d)[kBinAhead], uint32_t jb) {
#pragma unroll
        for (int k = 0; k < kBinAhead; ++k) d[k] = gload(sf, min(jb + k * 64 + lane, j1 - 1));
    };
    // Lanes of the set whose entry (inside the chunk) meets the group, and
    // their footprints and Gaussian indices.  Every lane issues the two loads
    // through a buffer resource of the set's 64 entries; the other lanes'
    // offsets lie past its range, so they read nothing from memory, and the
    // loads stay unconditional for the compiler's load-counter waits.
    auto pick = [&](const uint32_t (&d)[kBinAhead], uint64_t (&m)[kBinAhead], uint4 (&r)[kBinAhead],
                    uint32_t (&g)[kBinAhead], uint32_t jb) {
#pragma unroll
        for (int k = 0; k < kBinAhead; ++k) {
            const uint32_t base = __builtin_amdgcn_readfirstlane(jb + k * 64);
            const uint32_t nv = j1 > base ? j1 - base : 0u;
            const uint64_t in_chunk = nv >= 64 ? ~0ull : (1ull << nv) - 1ull;
            m[k] = __ballot(span_meets(d[k], gx, gy)) & in_chunk;
            const bool mine = (m[k] >> lane) & 1ull;
            const __amdgpu_buffer_rsrc_t br =
                __builtin_amdgcn_make_buffer_rsrc((void*)(rf + base), 0, 64 * 16, kBufferWord3);
            const __amdgpu_buffer_rsrc_t bo =
                __builtin_amdgcn_make_buffer_rsrc((void*)(of + base), 0, 64 * 4, kBufferWord3);
            const auto v = __builtin_amdgcn_raw_buffer_load_b128(br, mine ? lane * 16u : 64u * 16u, 0, 0);
            r[k] = make_uint4(v[0], v[1], v[2], v[3]);
            g[k] = __builtin_amdgcn_raw_buffer_load_b32(bo, mine ? lane * 4u : 64u * 4u, 0, 0);
        }
    };
    // Write the staged appends of every lane to its run, kStageTiles tiles
    // per store (lane = tile q + lane / kStageDepth, append lane % kStageDepth),
    // the stage reads of kFlushAhead stores ahead of their stores.  The flush ends
    // with every LDS operation complete (s_waitcnt lgkmcnt(0)), so the visit
    // loop that resumes waits for none of them.
    auto flush = [&]() {
        const uint32_t nst = (uint32_t)(sp - s_lane) / kStagePitch;
        const uint32_t i = lane % kStageDepth;
        for (uint32_t q0 = 0; q0 < 64; q0 += kFlushAhead * kStageTiles) {
            uint32_t n[kFlushAhead], s0[kFlushAhead], v[kFlushAhead];
#pragma unroll
            for (int u = 0; u < kFlushAhead; ++u) {
                const uint32_t q = q0 + u * kStageTiles + lane / kStageDepth;
                n[u] = __shfl(nst, (int)q);
                s0[u] = __shfl(slot, (int)q);
                v[u] = s_stage[i * kStagePitch + q];
            }
#pragma unroll
            for (int u = 0; u < kFlushAhead; ++u)
                if (i < n[u]) pair_g[s0[u] + i] = v[u];
        }
        slot += nst;
        sp = s_lane;
        __builtin_amdgcn_s_waitcnt(kWaitLgkm0);
    };
    // The last flush: with few appends per tile, one store per stage row
    // (each lane its own tile) takes fewer stores than one per kStageTiles
    // tiles.
    auto flush_last = [&]() {
        const uint32_t nst = (uint32_t)(sp - s_lane) / kStagePitch;
        uint32_t top = 0;  // most appends any lane holds
#pragma unroll
        for (uint32_t bit = kStageDepth; bit; bit >>= 1)
            if (__ballot(nst >= top + bit)) top += bit;
        if (top > kStageDepth / 2) {
            flush();
            return;
        }
        for (uint32_t r = 0; r < top; ++r)
            if (r < nst) pair_g[slot + r] = s_lane[r * kStagePitch];
    };
    // the picked entries in depth order, one at a time
    auto visit = [&](const uint64_t (&m)[kBinAhead], const uint4 (&r)[kBinAhead], const uint32_t (&g)[kBinAhead]) {
#pragma unroll
        for (int k = 0; k < kBinAhead; ++k) {
            uint64_t mm = m[k];
            while (mm) {
                const int p = __builtin_ctzll(mm);
                mm ^= 1ull << p;
                const uint32_t bx = __builtin_amdgcn_readlane(r[k].x, p);
                const uint32_t bz = __builtin_amdgcn_readlane(r[k].z, p), bw = __builtin_amdgcn_readlane(r[k].w, p);
                const uint32_t gp = __builtin_amdgcn_readlane(g[k], p);
                const uint32_t dx = lx - (bx & 0x7FFFu), dy = ly - (bx >> 16);  // wrap left of / above the box
                // the coverage-mask test, replaced below for a larger box
                const uint64_t mask = (uint64_t)bw << 32 | bz;
                bool hit = ((dx | dy) < kMaskSide) & (((mask >> ((dy * kMaskSide + dx) & 63u)) & 1u) != 0);
                if (!(bx & kMaskFlag)) {  // uniform branch
                    const Footprint fp(make_uint4(bx, __builtin_amdgcn_readlane(r[k].y, p), bz, bw));
                    int a, e;
                    fp.row(dy, a, e);
                    hit = valid & (dy < fp.h()) & ((int)lx >= a) & ((int)lx < e);
                }
                // every lane writes: a lane without a hit writes to the spare
                // row past its column's last, and its pointer stays
                *(hit ? sp : s_end) = gp;
                sp += hit ? kStagePitch : 0u;
                if (__ballot(sp == s_end)) flush();
            }
        }
    };
    uint32_t da[kBinAhead], db[kBinAhead];
    uint64_t ma[kBinAhead], mb[kBinAhead];
    uint4 ra[kBinAhead], rb[kBinAhead];
    uint32_t ga[kBinAhead], gb[kBinAhead];
    // The scheduling barriers keep the loads in the order written, so that
    // the compiler's load-counter waits leave the later sets in flight.
    load_spans(da, j0);
    load_spans(db, j0 + kSet);
    __builtin_amdgcn_sched_barrier(0);
    pick(da, ma, ra, ga, j0);
    __builtin_amdgcn_sched_barrier(0);
    load_spans(da, j0 + 2 * kSet);
    __builtin_amdgcn_sched_barrier(0);
    // Sets alternate between the a and b registers without copies.  The loop
    // has no exit in the middle (a set past the chunk picks nothing), for the
    // same reason.
    for (uint32_t j = j0; j < j1; j += 2 * kSet) {
        pick(db, mb, rb, gb, j + kSet);
        __builtin_amdgcn_sched_barrier(0);
        load_spans(db, j + 3 * kSet);
        __builtin_amdgcn_sched_barrier(0);
        visit(ma, ra, ga);
        pick(da, ma, ra, ga, j + 2 * kSet);
        __builtin_amdgcn_sched_barrier(0);
        load_spans(da, j + 4 * kSet);
        __builtin_amdgcn_sched_barrier(0);
        visit(mb, rb, gb);
    }
    flush_last();
}

// Per tile, exclusive prefix over the chunks (in place) and the tile's total.
// A block holds 64 tiles of one frame and ns waves (1 <= ns <= kScanSlices);
// wave s takes the s-th run of consecutive chunks, so each lane walks
// nch / ns rows instead of all nch.  With several runs each wave first sums
// its run, the runs' sums of one tile are prefixed through LDS, and each wave
// then rewrites its run as exclusive prefixes from its start; one run is
// rewritten in a single pass.  Rows are read coalesced (64 tiles of one chunk
// per wave load), eight at a time.
constexpr uint32_t kScanSlices = 8;

__global__ __launch_bounds__(64 * kScanSlices) void k_tile_colscan(const FrameDev* __restrict__ tab, BlockMap qm,
                                                                   uint32_t ns, uint32_t* __restrict__ cnt,
                                                                   uint32_t* __restrict__ ttot)
{
    __shared__ uint32_t s_sum[kScanSlices][64];
    const int f = frame_of_block(qm, blockIdx.x);
    const FrameDev& F = tab[f];
    const uint32_t lane = threadIdx.x & 63, sl = threadIdx.x >> 6;
    const uint32_t t = (blockIdx.x - qm.start[f]) * 64 + lane;
    const uint32_t T = F.tiles_x * F.tiles_y;
    const uint32_t nch = F.nch, per = (nch + ns - 1) / ns;
    const uint32_t c0 = min(nch, sl * per), c1 = min(nch, c0 + per);
    uint32_t* p = cnt + F.m0 + t;
    uint32_t run = 0;
    if (ns > 1) {  // uniform over the block
        uint32_t sum = 0;
        if (t < T) {
            uint32_t c = c0;
            for (; c + 8 <= c1; c += 8) {
                uint32_t v[8];
#pragma unroll
                for (int k = 0; k < 8; ++k) v[k] = p[(size_t)(c + k) * T];
#pragma unroll
                for (int k = 0; k < 8; ++k) sum += v[k];
            }
            for (; c < c1; ++c) sum += p[(size_t)c * T];
        }
        s_sum[sl][lane] = sum;
        __syncthreads();
        for (uint32_t q = 0; q < sl; ++q) run += s_sum[q][lane];
    }
    if (t >= T) return;
    uint32_t c = c0;
    for (; c + 8 <= c1; c += 8) {
        uint32_t v[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) v[k] = p[(size_t)(c + k) * T];
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            p[(size_t)(c + k) * T] = run;
            run += v[k];
        }
    }
    for (; c < c1; ++c) {
        const uint32_t v = p[(size_t)c * T];
        p[(size_t)c * T] = run;
        run += v;
    }
    if (sl == ns - 1) ttot[F.t0 + t] = run;
}

// Tile ranges from the scanned tile totals: tile t of frame f starts after
// the pairs of tiles 0 .. t-1 and ends where tile t + 1 starts (the last tile
// at the frame's pair count).
__global__ __launch_bounds__(256) void k_tile_ranges(const FrameDev* __restrict__ tab, BlockMap tm,
                                                     const uint32_t* __restrict__ counts,
                                                     const uint32_t* __restrict__ tstart,
                                                     uint2* __restrict__ ranges)
{
    const int f = frame_of_block(tm, blockIdx.x);
    const FrameDev& F = tab[f];
    const uint32_t t = (blockIdx.x - tm.start[f]) * 256 + threadIdx.x;
    const uint32_t T = F.tiles_x * F.tiles_y;
    if (t >= T) return;
    const uint32_t* cf = counts + f * SD7_CNT_WORDS;
    const uint32_t P = cf[SD7_CNT_PAIRS], pb = cf[SD7_CNT_PAIR_BASE];
    uint2 r = make_uint2(0u, 0u);
    if (P > 0) {
        const uint32_t* ts = tstart + F.t0;
        r.x = pb + ts[t] - ts[0];
        r.y = (t + 1 < T) ? pb + ts[t + 1] - ts[0] : pb + P;
    }
    ranges[F.t0 + t] = r;
}

// Calls of at most kFinishTiles tiles finish the counting binner's scalar
// steps in one block of 1024 lanes instead of five launches: the exclusive
// scan of the tile totals (in place, as the scan kernels leave it), the
// arena hand-out of k_setup_pairs (by its first wave) and every tile's range
// (as k_tile_ranges writes it, from the scanned totals and the frame's pair
// count and first slot, which the first wave passes on through LDS).
constexpr uint32_t kFinishThreads = 1024;
constexpr uint32_t kFinishPerThread = 16;
constexpr uint32_t kFinishTiles = kFinishThreads * kFinishPerThread;

__global__ __launch_bounds__(kFinishThreads) void k_tiles_finish(const FrameDev* __restrict__ tab, int nf,
                                                                 uint32_t ntiles, uint32_t capacity,
                                                                 uint32_t* __restrict__ ttot,
                                                                 uint32_t* __restrict__ counts,
                                                                 SortSeg* __restrict__ segs,
                                                                 SortTotals* __restrict__ tot,
                                                                 uint2* __restrict__ ranges)
{
    __shared__ uint32_t s_wave[kFinishThreads / 64];
    __shared__ uint32_t s_total;
    __shared__ uint2 s_frame[SD7_MAX_FRAMES];  // (pairs, first slot) per frame
    const uint32_t tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    // each lane's run of kFinishPerThread consecutive totals
    const uint32_t i0 = tid * kFinishPerThread;
    uint32_t v[kFinishPerThread], sum = 0;
#pragma unroll
    for (uint32_t k = 0; k < kFinishPerThread; ++k) {
        v[k] = i0 + k < ntiles ? ttot[i0 + k] : 0u;
        sum += v[k];
    }
    // exclusive prefix of the runs' sums: within the wave, then over waves
    const uint32_t incl = wave_incl_scan(sum, lane);
    if (lane == 63) s_wave[wave] = incl;
    __syncthreads();
    if (wave == 0) {
        const uint32_t w = lane < kFinishThreads / 64 ? s_wave[lane] : 0u;
        const uint32_t wi = wave_incl_scan(w, lane);
        if (lane < kFinishThreads / 64) s_wave[lane] = wi - w;
        if (lane == kFinishThreads / 64 - 1) s_total = wi;
    }
    __syncthreads();
    uint32_t run = s_wave[wave] + incl - sum;
#pragma unroll
    for (uint32_t k = 0; k < kFinishPerThread; ++k) {
        if (i0 + k < ntiles) ttot[i0 + k] = run;
        run += v[k];
    }
    // the stores above are read back by the first wave (other lanes' runs)
    __threadfence_block();
    __syncthreads();
    if (wave == 0) {
        const uint2 fr = setup_pairs_wave(tab, nf, ntiles, true, ttot, s_total, capacity, counts, segs, tot, lane);
        if ((int)lane < nf) s_frame[lane] = fr;
    }
    __syncthreads();
    for (int f = 0; f < nf; ++f) {
        const FrameDev& F = tab[f];
        const uint32_t T = F.tiles_x * F.tiles_y;
        const uint2 fr = s_frame[f];
        const uint32_t* ts = ttot + F.t0;
        for (uint32_t t = tid; t < T; t += kFinishThreads) {
            uint2 r = make_uint2(0u, 0u);
            if (fr.x > 0) {
                r.x = fr.y + ts[t] - ts[0];
                r.y = (t + 1 < T) ? fr.y + ts[t + 1] - ts[0] : fr.y + fr.x;
            }
            ranges[F.t0 + t] = r;
        }
    }
}

}  // namespace sd7
