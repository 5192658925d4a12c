// Host side of lib7dgs: argument checks, workspace planning, frame tables and
// kernel launches behind the C ABI of include/sd7.h.  Built as one
// translation unit with the kernel files.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>

#include "common.h"
#include "slice.hip"
#include "agr.hip"
#include "project.hip"
#include "slice_project.hip"
#include "bin.hip"
#include "raster.hip"
#include "densify.hip"
#include "optim.hip"

using namespace sd7;

namespace {

thread_local char g_err[512] = "";

sd7_status fail(sd7_status code, const char* fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
    return code;
}

#define HIP_TRY(expr)                                                                     \
    do {                                                                                  \
        hipError_t e_ = (expr);                                                           \
        if (e_ != hipSuccess) return fail(SD7_EHIP, "%s: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

#define LAUNCH_CHECK(name)                                                               \
    do {                                                                                 \
        hipError_t e_ = hipGetLastError();                                               \
        if (e_ != hipSuccess) return fail(SD7_EHIP, "launch %s: %s", name, hipGetErrorString(e_)); \
    } while (0)

constexpr size_t kAlign = 256;
constexpr int kRing = 64;             // pinned staging slots for frame tables

// The workspace of sd7_render_static: one per device, held from the library's
// load until the process ends.  Host code never passes this name to a kernel
// or a copy (on the host it is only a stand-in for the symbol): sd7_create
// looks up its device address with hipGetSymbolAddress and keeps it in the
// context.
static __device__ __align__(256) unsigned char scratch[SD7_STATIC_WS_BYTES];
constexpr int kPersistentBlocks = 2048;

size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }
uint32_t ceil_div(uint64_t a, uint64_t b) { return (uint32_t)((a + b - 1) / b); }

// Offsets of the scratch sub-arrays (inside off_scratch .. bytes).
struct Scratch {
    size_t sk_a, sv_a, sk_b;         // depth sort ping-pong (keys a, vals a, keys b)
    size_t pt_a, pt_b, pg_b;         // radix tile sort: tile keys and ping-pong buffers
    size_t toff;                     // tile offsets (scan of tiles per sorted Gaussian)
    size_t dhist, dctr, dstat;       // its digit counts, tile counters, status words
    size_t srect;                    // footprints in depth order (counting binner)
    size_t sspan;                    // their tile-group spans (counting binner)
    size_t segs_all, segs_kept, segs_pairs;
    size_t tot_all, tot_kept, tot_pairs;
    size_t hist, partials, words;
};

struct Plan {
    sd7_layout L;
    Scratch S;
    uint32_t max_wt_depth, max_wt_pairs;
    size_t hist_entries, partial_entries;
    BlockMap gmap;   // blocks of 256 Gaussians per frame
    SceneGroups sgrp;  // frames sharing a scene; blocks of 256 Gaussians per group
    bool single_runs;  // every scene group has one frame
    uint32_t sblocks;
    BlockMap tmap;   // one block per tile
    uint32_t gblocks, tblocks;
    // counting binner (frames of at most kMaxCountTiles tiles)
    bool counting;
    bool onesweep;  // depth sort with one launch per digit (calls of few work tiles)
    uint32_t max_tiles;
    int64_t max_n;  // Gaussians of the largest frame
    uint32_t nch[SD7_MAX_FRAMES], m0[SD7_MAX_FRAMES];
    BlockMap cmap;   // one block (wave) per (frame, chunk, tile group)
    BlockMap kmap;   // one block per (frame, chunk)
    uint32_t kblocks;
    BlockMap rmap;   // blocks of 256 tiles per frame
    BlockMap qmap;   // blocks of 64 tiles per frame
    uint32_t cblocks, rblocks, qblocks;
    size_t matrix_entries;
    size_t cnt;      // workspace offset of the count matrix
    size_t ttot;     // workspace offset of the per-tile totals (then their scan)
};

constexpr uint32_t kOneSweepTiles = 512;
constexpr uint32_t kRasterMaskedTiles = 4096;  // tiles of a call above which the compositing masks its blends
constexpr uint32_t kRasterBandTiles = 256;     // tiles of a call up to which each band gets a wave
constexpr uint32_t kScanSplitTiles = 16384;  // tiles of a call up to which the column scan splits its chunks  // depth-sort work tiles up to which a call sorts one launch per digit
constexpr uint64_t kBinWaves = 131072; // (chunk, group) waves the counting binner aims for per call
constexpr uint64_t kMaxChunks = 512;   // chunks per frame (the depth of the per-tile column scan)
constexpr size_t kMaxMatrix = (size_t)1 << 28;  // count-matrix entries of one call

// Binning chunks per frame: enough (chunk, group) waves over the call to fill
// the chip, at most kMaxChunks, and no more than one per 256 Gaussians (per 64
// in frames of at most 256 tiles, where a chunk's row of the count matrix
// costs little and a few long chunks would leave the placement waves walking
// their entries one after another).  The kernels cut the kept Gaussians (a
// count known on the device) into this many chunks.
uint32_t chunk_count(int64_t n, uint32_t groups, uint32_t tiles, int nf)
{
    if (n <= 0) return 0;
    const uint64_t per = (uint64_t)nf * groups;
    uint64_t nch = std::min<uint64_t>(std::max<uint64_t>(1, (kBinWaves + per - 1) / per), kMaxChunks);
    const uint64_t least = tiles <= 256 ? 64 : 256;
    return (uint32_t)std::min<uint64_t>(nch, ((uint64_t)n + least - 1) / least);
}

sd7_status make_plan(const sd7_frame* fr, int nf, int64_t cap, Plan& P, bool need_bwd)
{
    if (!fr) return fail(SD7_EINVAL, "frames is NULL");
    if (nf < 1 || nf > SD7_MAX_FRAMES) return fail(SD7_EINVAL, "nf=%d outside [1, %d]", nf, SD7_MAX_FRAMES);
    if (cap < 0 || cap >= (int64_t)1 << 31) return fail(SD7_EINVAL, "pair_capacity=%lld outside [0, 2^31)", (long long)cap);
    std::memset(&P, 0, sizeof(P));
    sd7_layout& L = P.L;
    L.nframes = nf;
    L.pair_capacity = cap;
    int64_t ntot = 0, ttot = 0;
    uint32_t max_tiles = 1;
    uint64_t wt_depth = 0;
    P.gmap.nf = nf;
    P.tmap.nf = nf;
    for (int f = 0; f < nf; ++f) {
        const sd7_frame& F = fr[f];
        const int64_t n = F.scene.n;
        if (n < 0 || n >= (int64_t)1 << 31) return fail(SD7_EINVAL, "frame %d: n=%lld outside [0, 2^31)", f, (long long)n);
        if (n > 0 && (!F.scene.mu_p || !F.scene.mu_t || !F.scene.mu_d || !F.scene.L || !F.scene.alpha || !F.scene.sh))
            return fail(SD7_EINVAL, "frame %d: NULL scene array", f);
        const int W = F.view.W, H = F.view.H;
        if (W < 1 || H < 1 || W > SD7_MAX_DIM || H > SD7_MAX_DIM)
            return fail(SD7_EINVAL, "frame %d: W=%d H=%d outside [1, %d]", f, W, H, SD7_MAX_DIM);
        if (!F.image || !F.final_T || !F.last) return fail(SD7_EINVAL, "frame %d: NULL image/final_T/last", f);
        if (!(F.view.fx > 0.f) || !(F.view.fy > 0.f)) return fail(SD7_EINVAL, "frame %d: focal length must be > 0", f);
        if (need_bwd && (!F.dL_dimage || !F.grad.mu_p || !F.grad.mu_t || !F.grad.mu_d || !F.grad.L ||
                         !F.grad.alpha || !F.grad.sh))
            return fail(SD7_EINVAL, "frame %d: NULL dL_dimage or gradient array", f);
        const uint32_t tx = ceil_div(W, kTile), ty = ceil_div(H, kTile);
        L.g0[f] = ntot;
        L.tile0[f] = ttot;
        P.gmap.start[f] = P.gblocks;
        P.tmap.start[f] = P.tblocks;
        P.gblocks += ceil_div(n, kBlock);
        P.tblocks += tx * ty;
        ntot += n;
        ttot += (int64_t)tx * ty;
        max_tiles = std::max(max_tiles, tx * ty);
        P.max_n = std::max(P.max_n, n);
        wt_depth += ceil_div(n, kSortItems);
        const uint32_t groups = ceil_div(tx, kGroup) * ceil_div(ty, kGroup);
        P.nch[f] = chunk_count(n, groups, tx * ty, nf);
        P.m0[f] = (uint32_t)std::min<size_t>(P.matrix_entries, UINT32_MAX);
        P.cmap.start[f] = P.cblocks;
        P.kmap.start[f] = P.kblocks;
        P.rmap.start[f] = P.rblocks;
        P.qmap.start[f] = P.qblocks;
        P.kblocks += P.nch[f];
        P.cblocks += P.nch[f] * groups;
        P.rblocks += ceil_div(tx * ty, 256);
        P.qblocks += ceil_div(tx * ty, 64);
        P.matrix_entries += (size_t)P.nch[f] * tx * ty;
    }
    P.gmap.start[nf] = P.gblocks;
    // scene groups (same parameter arrays and n), in order of first appearance
    {
        int owner[SD7_MAX_FRAMES], head[SD7_MAX_FRAMES];
        int ng = 0;
        for (int f = 0; f < nf; ++f) {
            const sd7_scene& A = fr[f].scene;
            owner[f] = -1;
            for (int g = 0; g < ng && owner[f] < 0; ++g) {
                const sd7_scene& B = fr[head[g]].scene;
                if (A.n == B.n && A.mu_p == B.mu_p && A.mu_t == B.mu_t && A.mu_d == B.mu_d && A.L == B.L &&
                    A.alpha == B.alpha && A.sh == B.sh)
                    owner[f] = g;
            }
            if (owner[f] < 0) {
                head[ng] = f;
                owner[f] = ng++;
            }
        }
        int q = 0;
        uint64_t units = 0;
        for (int g = 0; g < ng; ++g) {
            P.sgrp.first[g] = (uint8_t)q;
            P.sgrp.start[g] = (uint32_t)std::min<uint64_t>(units, UINT32_MAX);
            const int q0 = q;
            for (int f = 0; f < nf; ++f)
                if (owner[f] == g) P.sgrp.frame[q++] = (uint8_t)f;
            units += (uint64_t)ceil_div(fr[head[g]].scene.n, kBlock) * (uint64_t)(q - q0);
        }
        P.sgrp.first[ng] = (uint8_t)q;
        P.sgrp.start[ng] = (uint32_t)std::min<uint64_t>(units, UINT32_MAX);
        P.sgrp.ng = ng;
        P.single_runs = ng == nf;
        // whole rounds of resident blocks, equal shares of the units
        const uint64_t rounds = std::max<uint64_t>(1, units / ((uint64_t)kSliceResident * kSliceUnitsPerBlock));
        P.sblocks = (uint32_t)std::min<uint64_t>(units, kSliceResident * rounds);
    }
    P.tmap.start[nf] = P.tblocks;
    P.cmap.start[nf] = P.cblocks;
    P.kmap.start[nf] = P.kblocks;
    P.rmap.start[nf] = P.rblocks;
    P.qmap.start[nf] = P.qblocks;
    P.cmap.nf = P.kmap.nf = P.rmap.nf = P.qmap.nf = nf;
    P.max_tiles = max_tiles;
    P.counting = max_tiles <= kMaxCountTiles && P.matrix_entries <= kMaxMatrix;
    if (ntot >= (int64_t)1 << 31) return fail(SD7_EINVAL, "total Gaussians %lld >= 2^31", (long long)ntot);
    if (ttot >= (int64_t)1 << 31) return fail(SD7_EINVAL, "total tiles %lld >= 2^31", (long long)ttot);
    if (cap + (int64_t)nf * kSortItems >= (int64_t)1 << 31) return fail(SD7_EINVAL, "pair capacity too large");
    L.n_total = ntot;
    L.tiles_total = ttot;
    int bits = 0;
    while ((1u << bits) < max_tiles) ++bits;
    L.tile_sort_passes = std::max(1, (bits + 7) / 8);
    P.max_wt_depth = (uint32_t)wt_depth;
    P.onesweep = P.max_wt_depth <= kOneSweepTiles;
    P.max_wt_pairs = ceil_div(cap, kSortItems) + nf;

    const size_t N = (size_t)ntot, T = (size_t)ttot, C = (size_t)cap;
    size_t off = 0;
    auto take = [&](size_t bytes) { const size_t o = off; off = align_up(off + bytes); return o; };
    L.off_table = take(sizeof(FrameDev) * nf);
    L.off_counts = take(sizeof(uint32_t) * SD7_CNT_WORDS * nf);
    L.off_mu_c = take(4 * 3 * N);
    L.off_cov_c = take(4 * 6 * N);
    L.off_alpha_c = take(4 * N);
    L.off_splat = take(4 * kSplatFloats * N);
    L.off_rect = take(16 * N);
    L.off_depth_key = take(4 * N);
    L.off_order = take(4 * N);
    L.off_pair_g = take(4 * C);
    L.off_ranges = take(8 * T);
    L.off_d_splat = take(4 * 9 * N);
    L.off_d_mu_c = take(4 * 3 * N);
    L.off_d_cov_c = take(4 * 6 * N);
    L.off_d_alpha_c = take(4 * N);
    L.off_scratch = off;
    Scratch& S = P.S;
    S.sk_a = take(4 * N);
    S.sv_a = take(4 * N);
    S.sk_b = take(4 * N);
    // tile keys and ping-pong buffers of the radix tile sort (fallback binner)
    const size_t CR = P.counting ? 0 : C;
    S.pt_a = take(4 * CR);
    S.pt_b = take(4 * CR);
    S.pg_b = take(4 * CR);
    S.toff = take(4 * (P.counting ? 0 : N + 16));
    S.srect = take(16 * (P.counting ? N : 0));
    S.sspan = take(4 * (P.counting ? N : 0));
    S.segs_all = take(sizeof(SortSeg) * nf);
    S.segs_kept = take(sizeof(SortSeg) * nf);
    S.segs_pairs = take(sizeof(SortSeg) * nf);
    S.tot_all = take(sizeof(SortTotals));
    S.tot_kept = take(sizeof(SortTotals));
    S.tot_pairs = take(sizeof(SortTotals));
    P.hist_entries = 256 * (size_t)std::max(P.onesweep ? 0u : P.max_wt_depth, P.counting ? 0u : P.max_wt_pairs);
    S.hist = take(4 * P.hist_entries);
    // small calls' depth sort: digit counts [nf][4][256] and tile counters [4]
    // (zeroed by k_setup_depth), status words [4][max_wt_depth][256] (zeroed
    // by k_depth_hist)
    S.dhist = take(P.onesweep ? 4 * 1024 * (size_t)nf : 0);
    S.dctr = take(P.onesweep ? 4 * 4 : 0);
    S.dstat = take(P.onesweep ? 4 * 4 * 256 * (size_t)P.max_wt_depth : 0);
    const size_t mat = P.counting ? P.matrix_entries : 0;
    P.cnt = take(4 * mat);
    P.ttot = take(4 * (P.counting ? T + 4 : 0));
    P.partial_entries = std::max(std::max(P.hist_entries, N), mat) / kScanItems + 4;
    S.partials = take(4 * P.partial_entries);
    S.words = take(4 * 64);
    L.bytes = off;
    return SD7_OK;
}

}  // namespace

// Stages timed under SD7_PROFILE=1, in the order sd7_profile_read reports them.
enum ProfStage { kPSlice, kPProject, kPSliceProject, kPBin, kPRaster, kPRasterBwd, kPProjectBwd, kPSliceBwd,
                 kPStages };
const char* const kProfNames[kPStages] = {"slice", "project", "slice_project", "bin", "rasterize",
                                          "rasterize_backward", "project_backward", "slice_backward"};
constexpr int kProfSlots = 256;  // (start, end) event pairs in flight

struct sd7_ctx {
    int device = 0;
    char* scratch = nullptr;     // device address of this device's `scratch` array
    char* ring = nullptr;        // pinned host staging for frame tables
    size_t slot_bytes = 0;
    hipEvent_t ev[kRing];
    bool used[kRing];
    int next = 0;
    std::mutex mu;
    // per-stage timing (SD7_PROFILE=1 at creation): event pairs in a ring,
    // slots [pf_head, pf_head + pf_n) recorded and not yet read
    bool profile = false;
    hipEvent_t pf_start[kProfSlots], pf_end[kProfSlots];
    int pf_stage[kProfSlots];
    int pf_head = 0, pf_n = 0;
    uint64_t pf_calls[kPStages] = {};
    double pf_total[kPStages] = {}, pf_max[kPStages] = {};
    std::mutex pf_mu;
};

namespace {

// Frame table -> workspace (through a pinned staging slot, stream ordered).
sd7_status upload_table(sd7_ctx* ctx, const sd7_frame* fr, int nf, const Plan& P, char* ws, hipStream_t st)
{
    std::lock_guard<std::mutex> lock(ctx->mu);
    const int slot = ctx->next;
    ctx->next = (ctx->next + 1) % kRing;
    if (ctx->used[slot]) HIP_TRY(hipEventSynchronize(ctx->ev[slot]));
    FrameDev* tab = reinterpret_cast<FrameDev*>(ctx->ring + (size_t)slot * ctx->slot_bytes);
    for (int f = 0; f < nf; ++f) {
        const sd7_frame& F = fr[f];
        FrameDev& D = tab[f];
        std::memset(&D, 0, sizeof(D));
        D.mu_p = F.scene.mu_p; D.mu_t = F.scene.mu_t; D.mu_d = F.scene.mu_d;
        D.L = F.scene.L; D.alpha = F.scene.alpha; D.sh = F.scene.sh;
        D.image = F.image; D.final_T = F.final_T; D.last = F.last; D.dL_dimage = F.dL_dimage;
        D.g_mu_p = F.grad.mu_p; D.g_mu_t = F.grad.mu_t; D.g_mu_d = F.grad.mu_d;
        D.g_L = F.grad.L; D.g_alpha = F.grad.alpha; D.g_sh = F.grad.sh;
        D.g_lambda = F.grad.lambda;
        D.d_mode = F.view.d_per_gaussian ? 1u : 0u;
        D.ncontrib = F.ncontrib;
        D.agr = F.scene.agr;
        D.n = (uint32_t)F.scene.n;
        D.g0 = (uint32_t)P.L.g0[f];
        D.W = (uint32_t)F.view.W;
        D.H = (uint32_t)F.view.H;
        D.tiles_x = ceil_div(D.W, kTile);
        D.tiles_y = ceil_div(D.H, kTile);
        D.t0 = (uint32_t)P.L.tile0[f];
        D.nch = P.nch[f];
        D.m0 = P.m0[f];
        D.keep_sliced = (F.outputs & SD7_OUT_SLICED) || F.grad.L ? 1u : 0u;
        std::memcpy(D.R, F.view.R_wc, sizeof(D.R));
        std::memcpy(D.c, F.view.c, sizeof(D.c));
        D.fx = F.view.fx; D.fy = F.view.fy; D.cx = F.view.cx; D.cy = F.view.cy;
        D.t = F.view.t;
        std::memcpy(D.d, F.view.d, sizeof(D.d));
        D.lambda_t = F.view.lambda_t; D.lambda_d = F.view.lambda_d;
        D.limx = kJClamp * (0.5f * (float)F.view.W) / F.view.fx;
        D.limy = kJClamp * (0.5f * (float)F.view.H) / F.view.fy;
        std::memcpy(D.bg, F.view.bg, sizeof(D.bg));
    }
    HIP_TRY(hipMemcpyAsync(ws + P.L.off_table, tab, sizeof(FrameDev) * nf, hipMemcpyHostToDevice, st));
    HIP_TRY(hipEventRecord(ctx->ev[slot], st));
    ctx->used[slot] = true;
    return SD7_OK;
}

struct Call {
    Plan P;
    sd7_ctx* ctx = nullptr;
    char* ws;
    hipStream_t st;
    const FrameDev* tab;
    uint32_t* counts;
    bool count;  // some frame asks for per-pixel contributor counts
    bool agr;    // some frame's scene has AGR weights
    template <class T>
    T* at(size_t off) const { return reinterpret_cast<T*>(ws + off); }
};

// Plan the call and set up its launch state (no device work).
sd7_status prepare(sd7_ctx* ctx, const sd7_frame* fr, int nf, int64_t cap, void* ws, size_t ws_bytes,
                   sd7_stream stream, Call& c, bool need_bwd)
{
    if (!ctx) return fail(SD7_EINVAL, "ctx is NULL");
    if (!ws) return fail(SD7_EINVAL, "workspace is NULL");
    sd7_status s = make_plan(fr, nf, cap, c.P, need_bwd);
    if (s != SD7_OK) return s;
    if (ws_bytes < c.P.L.bytes)
        return fail(SD7_EWORKSPACE, "workspace has %zu bytes, %zu needed", ws_bytes, c.P.L.bytes);
    if (reinterpret_cast<uintptr_t>(ws) % kAlign) return fail(SD7_EINVAL, "workspace not 256-byte aligned");
    HIP_TRY(hipSetDevice(ctx->device));
    c.ws = static_cast<char*>(ws);
    c.st = static_cast<hipStream_t>(stream);
    c.tab = c.at<FrameDev>(c.P.L.off_table);
    c.counts = c.at<uint32_t>(c.P.L.off_counts);
    c.count = false;
    c.agr = false;
    for (int f = 0; f < nf; ++f) {
        c.count = c.count || fr[f].ncontrib != nullptr;
        c.agr = c.agr || fr[f].scene.agr != nullptr;
    }
    if (need_bwd && c.agr) return fail(SD7_EINVAL, "the reverse calls do not support AGR scenes");
    return SD7_OK;
}

sd7_status begin(sd7_ctx* ctx, const sd7_frame* fr, int nf, int64_t cap, void* ws, size_t ws_bytes,
                 sd7_stream stream, Call& c, bool need_bwd)
{
    g_err[0] = 0;
    sd7_status s = prepare(ctx, fr, nf, cap, ws, ws_bytes, stream, c, need_bwd);
    if (s != SD7_OK) return s;
    c.ctx = ctx;
    return upload_table(ctx, fr, nf, c.P, c.ws, c.st);
}

// Adds a finished (start, end) pair to its stage's totals and frees the
// oldest slot (the caller holds pf_mu).
sd7_status profile_retire(sd7_ctx* ctx)
{
    const int k = ctx->pf_head;
    HIP_TRY(hipEventSynchronize(ctx->pf_end[k]));
    float ms = 0.f;
    HIP_TRY(hipEventElapsedTime(&ms, ctx->pf_start[k], ctx->pf_end[k]));
    const int st = ctx->pf_stage[k];
    ctx->pf_calls[st] += 1;
    ctx->pf_total[st] += ms;
    ctx->pf_max[st] = std::max(ctx->pf_max[st], (double)ms);
    ctx->pf_head = (k + 1) % kProfSlots;
    ctx->pf_n -= 1;
    return SD7_OK;
}

// Runs one stage; with profiling on, between two events on the call's
// stream (the oldest pair is read first when every slot is in flight).
template <class F>
sd7_status timed(const Call& c, ProfStage stage, F&& run)
{
    sd7_ctx* ctx = c.ctx;
    if (!ctx || !ctx->profile) return run();
    int k;
    {
        std::lock_guard<std::mutex> lock(ctx->pf_mu);
        if (ctx->pf_n == kProfSlots) {
            const sd7_status s = profile_retire(ctx);
            if (s != SD7_OK) return s;
        }
        k = (ctx->pf_head + ctx->pf_n) % kProfSlots;
        ctx->pf_n += 1;
        ctx->pf_stage[k] = stage;
        HIP_TRY(hipEventRecord(ctx->pf_start[k], c.st));
    }
    const sd7_status s = run();
    HIP_TRY(hipEventRecord(ctx->pf_end[k], c.st));
    return s;
}

sd7_status fill(const Call& c, void* p, size_t count, uint32_t value)
{
    if (count == 0) return SD7_OK;
    const uint32_t blocks = std::min<uint32_t>(ceil_div(count, 256), 4096);
    k_fill_u32<<<blocks, 256, 0, c.st>>>(static_cast<uint32_t*>(p), count, value);
    LAUNCH_CHECK("k_fill_u32");
    return SD7_OK;
}

// Exclusive scan in place; the length is host-known (len_dev null) or read on
// the device; the grand total goes to *total_out when asked for.  Up to
// kScanCarryTiles work tiles (by max_len) the down-sweep adds up the tile
// sums itself; longer scans take a spine pass between.
// part: at least max_len / kScanItems + 4 entries.
sd7_status scan_with(hipStream_t st, uint32_t* part, uint32_t* data, uint32_t len_host, const uint32_t* len_dev,
                     uint32_t max_len, uint32_t* total_out)
{
    const uint32_t tiles = ceil_div(max_len, kScanItems);
    const uint32_t blocks = std::max(1u, std::min<uint32_t>(tiles, kPersistentBlocks));
    k_scan_reduce<<<blocks, 256, 0, st>>>(data, len_host, len_dev, part);
    LAUNCH_CHECK("k_scan_reduce");
    if (tiles <= kScanCarryTiles) {
        k_scan_down<true><<<blocks, 256, 0, st>>>(data, data, len_host, len_dev, part, total_out);
        LAUNCH_CHECK("k_scan_down");
        return SD7_OK;
    }
    k_scan_spine<<<1, 1024, 0, st>>>(part, len_host, len_dev, total_out);
    LAUNCH_CHECK("k_scan_spine");
    k_scan_down<false><<<blocks, 256, 0, st>>>(data, data, len_host, len_dev, part, nullptr);
    LAUNCH_CHECK("k_scan_down");
    return SD7_OK;
}

sd7_status scan(const Call& c, uint32_t* data, uint32_t len_host, const uint32_t* len_dev, uint32_t max_len,
                uint32_t* total_out)
{
    return scan_with(c.st, c.at<uint32_t>(c.P.S.partials), data, len_host, len_dev, max_len, total_out);
}

// Pruning workspace: keep flags [n], their exclusive scan [n], scan partials.
struct PruneWs {
    size_t keep, pos, part, bytes;
};
PruneWs prune_ws(int64_t n)
{
    PruneWs w;
    size_t off = 0;
    w.keep = off; off = align_up(off + 4 * (size_t)n);
    w.pos = off;  off = align_up(off + 4 * (size_t)n);
    w.part = off; off = align_up(off + 4 * ((size_t)n / kScanItems + 8));
    w.bytes = off;
    return w;
}

sd7_status radix_pass(const Call& c, bool first, const uint32_t* kin, const uint32_t* vin, uint32_t* kout,
                      uint32_t* vout, const SortSeg* segs, const SortTotals* tot, uint32_t max_wt, int shift)
{
    if (max_wt == 0) return SD7_OK;
    uint32_t* hist = c.at<uint32_t>(c.P.S.hist);
    const int nf = c.P.L.nframes;
    const uint32_t blocks = std::min<uint32_t>(max_wt, kPersistentBlocks);
    if (first) k_radix_hist<true><<<blocks, 256, 0, c.st>>>(kin, segs, nf, tot, shift, hist);
    else k_radix_hist<false><<<blocks, 256, 0, c.st>>>(kin, segs, nf, tot, shift, hist);
    LAUNCH_CHECK("k_radix_hist");
    sd7_status s = scan(c, hist, 0, &tot->hist_len, 256u * max_wt, nullptr);
    if (s != SD7_OK) return s;
    if (first) k_radix_scatter<true><<<blocks, 256, 0, c.st>>>(kin, vin, kout, vout, segs, nf, tot, shift, hist);
    else k_radix_scatter<false><<<blocks, 256, 0, c.st>>>(kin, vin, kout, vout, segs, nf, tot, shift, hist);
    LAUNCH_CHECK("k_radix_scatter");
    return SD7_OK;
}

sd7_status do_slice(const Call& c)
{
    const sd7_layout& L = c.P.L;
    sd7_status s = fill(c, c.counts, (size_t)SD7_CNT_WORDS * L.nframes, 0);
    if (s != SD7_OK || c.P.gblocks == 0) return s;
    k_slice<<<c.P.gblocks, kBlock, 0, c.st>>>(c.tab, c.P.gmap, c.at<float>(L.off_mu_c), c.at<float>(L.off_cov_c),
                                               c.at<float>(L.off_alpha_c), c.counts);
    LAUNCH_CHECK("k_slice");
    if (c.agr) {  // frames whose scene is refined first (k_slice skipped them)
        k_agr_slice<<<c.P.gblocks, kBlock, 0, c.st>>>(c.tab, c.P.gmap, c.at<float>(L.off_mu_c),
                                                       c.at<float>(L.off_cov_c), c.at<float>(L.off_alpha_c),
                                                       c.counts);
        LAUNCH_CHECK("k_agr_slice");
    }
    return SD7_OK;
}

sd7_status do_project(const Call& c)
{
    const sd7_layout& L = c.P.L;
    if (c.P.gblocks == 0) return SD7_OK;
    k_project<<<c.P.gblocks, kBlock, 0, c.st>>>(c.tab, c.P.gmap, c.at<float>(L.off_mu_c), c.at<float>(L.off_cov_c),
                                                 c.at<float>(L.off_alpha_c), c.at<float4>(L.off_splat),
                                                 c.at<uint4>(L.off_rect), c.at<uint32_t>(L.off_depth_key), c.counts);
    LAUNCH_CHECK("k_project");
    return SD7_OK;
}

// Slice + project over scene groups (bitwise the same outputs as do_slice
// followed by do_project).
sd7_status do_slice_project(const Call& c)
{
    const sd7_layout& L = c.P.L;
    if (c.agr) {  // refined parameters depend on t: nothing to share across frames
        sd7_status s = do_slice(c);
        return s != SD7_OK ? s : do_project(c);
    }
    sd7_status s = fill(c, c.counts, (size_t)SD7_CNT_WORDS * L.nframes, 0);
    if (s != SD7_OK || c.P.sblocks == 0) return s;
    auto launch = [&](auto block_kept) {
        k_slice_project<decltype(block_kept)::value><<<c.P.sblocks, kBlock, 0, c.st>>>(
            c.tab, c.P.sgrp, c.at<float>(L.off_mu_c), c.at<float>(L.off_cov_c), c.at<float>(L.off_alpha_c),
            c.at<float4>(L.off_splat), c.at<uint4>(L.off_rect), c.at<uint32_t>(L.off_depth_key), c.counts);
    };
    if (c.P.single_runs) launch(std::true_type{});
    else launch(std::false_type{});
    LAUNCH_CHECK("k_slice_project");
    return SD7_OK;
}

sd7_status do_bin(const Call& c)
{
    const sd7_layout& L = c.P.L;
    const Scratch& S = c.P.S;
    const int nf = L.nframes;
    sd7_status s;
    SortSeg* segs_all = c.at<SortSeg>(S.segs_all);
    SortSeg* segs_kept = c.at<SortSeg>(S.segs_kept);
    SortSeg* segs_pairs = c.at<SortSeg>(S.segs_pairs);
    SortTotals* tot_all = c.at<SortTotals>(S.tot_all);
    SortTotals* tot_kept = c.at<SortTotals>(S.tot_kept);
    SortTotals* tot_pairs = c.at<SortTotals>(S.tot_pairs);
    uint32_t* words = c.at<uint32_t>(S.words);
    // Depth sort: one block per frame where every frame's keys fit one block;
    // otherwise the segments, then four digit passes.  The one-launch-per-digit
    // sort's digit counts and tile counters start at zero (its status words
    // are zeroed by k_depth_hist).
    uint32_t* order = c.at<uint32_t>(L.off_order);
    const uint32_t* dkey = c.at<uint32_t>(L.off_depth_key);
    const bool small = c.P.max_n <= (int64_t)kSmallSortItems;
    const bool os = !small && c.P.onesweep && c.P.max_wt_depth;
    if (small) {
        k_depth_small<<<nf, kSmallSortThreads, 0, c.st>>>(c.tab, c.counts, dkey, order);
        LAUNCH_CHECK("k_depth_small");
    } else {
        k_setup_depth<<<1, 256, 0, c.st>>>(c.tab, nf, c.counts, segs_all, tot_all, segs_kept, tot_kept,
                                           os ? c.at<uint32_t>(S.dhist) : nullptr,
                                           os ? (uint32_t)((S.dstat - S.dhist) / 4) : 0u);
        LAUNCH_CHECK("k_setup_depth");
    }
    // digit passes: key_depth -> (a) -> (b) -> (a) -> (b = order)
    uint32_t* ka = c.at<uint32_t>(S.sk_a);
    uint32_t* va = c.at<uint32_t>(S.sv_a);
    uint32_t* kb = c.at<uint32_t>(S.sk_b);
    const uint32_t mw = c.P.max_wt_depth;
    if (small) {
        // sorted above
    } else if (os) {
        uint32_t* dh = c.at<uint32_t>(S.dhist);
        uint32_t* ctr = c.at<uint32_t>(S.dctr);
        uint32_t* stat = c.at<uint32_t>(S.dstat);
        const size_t sw = 256 * (size_t)mw;  // status words of one pass
        k_depth_hist<<<mw, 256, 0, c.st>>>(dkey, segs_all, nf, tot_all, dh, stat, sw);
        LAUNCH_CHECK("k_depth_hist");
        k_depth_pass<true, true><<<mw, 256, 0, c.st>>>(dkey, nullptr, ka, va, segs_all, nf, tot_all, 0, dh, stat,
                                                       ctr, c.counts);
        LAUNCH_CHECK("k_depth_pass");
        k_depth_pass<false, true><<<mw, 256, 0, c.st>>>(ka, va, kb, order, segs_kept, nf, tot_kept, 1, dh,
                                                        stat + sw, ctr + 1, c.counts);
        LAUNCH_CHECK("k_depth_pass");
        k_depth_pass<false, true><<<mw, 256, 0, c.st>>>(kb, order, ka, va, segs_kept, nf, tot_kept, 2, dh,
                                                        stat + 2 * sw, ctr + 2, c.counts);
        LAUNCH_CHECK("k_depth_pass");
        k_depth_pass<false, false><<<mw, 256, 0, c.st>>>(ka, va, nullptr, order, segs_kept, nf, tot_kept, 3, dh,
                                                         stat + 3 * sw, ctr + 3, c.counts);
        LAUNCH_CHECK("k_depth_pass");
    } else {
        if ((s = radix_pass(c, true, dkey, nullptr, ka, va, segs_all, tot_all, mw, 0)) != SD7_OK) return s;
        if ((s = radix_pass(c, false, ka, va, kb, order, segs_kept, tot_kept, mw, 8)) != SD7_OK) return s;
        if ((s = radix_pass(c, false, kb, order, ka, va, segs_kept, tot_kept, mw, 16)) != SD7_OK) return s;
        if ((s = radix_pass(c, false, ka, va, kb, order, segs_kept, tot_kept, mw, 24)) != SD7_OK) return s;
    }
    if (c.P.counting) {
        // counting binner: depth-sorted boxes -> [chunk][tile] counts -> per-tile
        // prefix over chunks and tile totals -> scan of the totals (which also
        // gives each frame's pair count) -> arena -> placement -> ranges
        uint32_t* cnt = c.at<uint32_t>(c.P.cnt);
        uint32_t* ttot = c.at<uint32_t>(c.P.ttot);
        uint4* srect = c.at<uint4>(S.srect);
        const uint32_t ttiles = (uint32_t)L.tiles_total;
        if (c.P.gblocks) {
            k_gather_boxes<<<c.P.gblocks, kBlock, 0, c.st>>>(c.tab, c.P.gmap, c.counts, order,
                                                             c.at<uint4>(L.off_rect), srect,
                                                             c.at<uint32_t>(S.sspan));
            LAUNCH_CHECK("k_gather_boxes");
        }
        if (c.P.kblocks) {
            k_tile_count<<<c.P.kblocks, 256, sizeof(uint32_t) * c.P.max_tiles, c.st>>>(c.tab, c.P.kmap, c.counts,
                                                                                      srect, cnt);
            LAUNCH_CHECK("k_tile_count");
        }
        {
            // several runs of chunks per tile where the call has too few
            // tiles to fill the chip with one lane each
            const uint32_t ns = c.P.tblocks <= kScanSplitTiles ? kScanSlices : 1;
            k_tile_colscan<<<c.P.qblocks, 64 * ns, 0, c.st>>>(c.tab, c.P.qmap, ns, cnt, ttot);
        }
        LAUNCH_CHECK("k_tile_colscan");
        // scan of the tile totals, arena, ranges: one block for calls of few
        // tiles (the ranges need only the scan and the arena)
        const bool one_block = ttiles <= kFinishTiles;
        if (one_block) {
            k_tiles_finish<<<1, kFinishThreads, 0, c.st>>>(c.tab, nf, ttiles, (uint32_t)L.pair_capacity, ttot,
                                                          c.counts, segs_pairs, tot_pairs,
                                                          c.at<uint2>(L.off_ranges));
            LAUNCH_CHECK("k_tiles_finish");
        } else {
            if ((s = fill(c, words, 1, 0)) != SD7_OK) return s;
            if ((s = scan(c, ttot, ttiles, nullptr, ttiles, words)) != SD7_OK) return s;
            k_setup_pairs<<<1, 64, 0, c.st>>>(c.tab, nf, ttiles, true, ttot, words, (uint32_t)L.pair_capacity,
                                              c.counts, segs_pairs, tot_pairs);
            LAUNCH_CHECK("k_setup_pairs");
        }
        if (c.P.cblocks) {
            k_group_place<<<c.P.cblocks, 64, 0, c.st>>>(c.tab, c.P.cmap, c.counts, order, srect,
                                                         c.at<uint32_t>(S.sspan), cnt, ttot,
                                                         c.at<uint32_t>(L.off_pair_g));
            LAUNCH_CHECK("k_group_place");
        }
        if (!one_block) {
            k_tile_ranges<<<c.P.rblocks, 256, 0, c.st>>>(c.tab, c.P.rmap, c.counts, ttot, c.at<uint2>(L.off_ranges));
            LAUNCH_CHECK("k_tile_ranges");
        }
        return SD7_OK;
    }
    // tiles per sorted Gaussian -> exclusive offsets
    uint32_t* toff = c.at<uint32_t>(S.toff);
    if (c.P.gblocks) {
        k_gather_ntiles<<<c.P.gblocks, kBlock, 0, c.st>>>(c.tab, c.P.gmap, c.counts, order,
                                                          c.at<uint4>(L.off_rect), toff);
        LAUNCH_CHECK("k_gather_ntiles");
    }
    const uint32_t ntot = (uint32_t)L.n_total;
    if ((s = fill(c, words, 1, 0)) != SD7_OK) return s;
    if (ntot && (s = scan(c, toff, ntot, nullptr, ntot, words)) != SD7_OK) return s;
    k_setup_pairs<<<1, 64, 0, c.st>>>(c.tab, nf, ntot, false, toff, words, (uint32_t)L.pair_capacity, c.counts,
                                      segs_pairs, tot_pairs);
    LAUNCH_CHECK("k_setup_pairs");
    if ((s = fill(c, c.at<uint32_t>(L.off_ranges), 2 * (size_t)L.tiles_total, 0)) != SD7_OK) return s;
    // emit so that the last tile-sort pass lands in the pair_g array
    uint32_t* pt_a = c.at<uint32_t>(S.pt_a);
    uint32_t* pg_a = c.at<uint32_t>(L.off_pair_g);
    uint32_t* pt_b = c.at<uint32_t>(S.pt_b);
    uint32_t* pg_b = c.at<uint32_t>(S.pg_b);
    const int passes = L.tile_sort_passes;
    uint32_t *ct = (passes & 1) ? pt_b : pt_a, *cg = (passes & 1) ? pg_b : pg_a;
    uint32_t *ot = (passes & 1) ? pt_a : pt_b, *og = (passes & 1) ? pg_a : pg_b;
    const uint32_t mwp = c.P.max_wt_pairs;
    if (L.pair_capacity > 0) {
        const uint32_t blocks = std::min<uint32_t>(mwp, kPersistentBlocks);
        k_emit<<<blocks, 256, 0, c.st>>>(c.tab, c.counts, order, c.at<uint4>(L.off_rect), toff, segs_pairs, nf,
                                         tot_pairs, ct, cg);
        LAUNCH_CHECK("k_emit");
        for (int p = 0; p < passes; ++p) {
            if ((s = radix_pass(c, false, ct, cg, ot, og, segs_pairs, tot_pairs, mwp, 8 * p)) != SD7_OK) return s;
            std::swap(ct, ot);
            std::swap(cg, og);
        }
        k_ranges<<<blocks, 256, 0, c.st>>>(c.tab, pt_a, segs_pairs, nf, tot_pairs, c.at<uint2>(L.off_ranges));
        LAUNCH_CHECK("k_ranges");
    }
    return SD7_OK;
}

sd7_status do_raster(const Call& c)
{
    const sd7_layout& L = c.P.L;
    const uint2* rg = c.at<uint2>(L.off_ranges);
    const uint32_t* pg = c.at<uint32_t>(L.off_pair_g);
    const float4* sp = c.at<float4>(L.off_splat);
    // 64-bit addressing where a frame's splat records span 4 GiB or more
    const bool wide = c.P.max_n > (int64_t)(UINT32_MAX / (4 * kSplatFloats));
    if (!c.count && c.P.tblocks <= kRasterBandTiles) {  // one wave per band of each tile
        if (wide)
            k_raster_bands<true><<<4 * c.P.tblocks, 64, 0, c.st>>>(c.tab, c.P.tmap, rg, pg, sp);
        else
            k_raster_bands<false><<<4 * c.P.tblocks, 64, 0, c.st>>>(c.tab, c.P.tmap, rg, pg, sp);
        LAUNCH_CHECK("k_raster_bands");
        return SD7_OK;
    }
    // masked blends where several tile waves share each SIMD
    const bool masked = c.P.tblocks > kRasterMaskedTiles;
    auto launch = [&](auto count, auto wide_c, auto masked_c) {
        k_raster<decltype(count)::value, decltype(wide_c)::value, decltype(masked_c)::value>
            <<<c.P.tblocks, 64, 0, c.st>>>(c.tab, c.P.tmap, rg, pg, sp);
    };
    auto with_masked = [&](auto count, auto wide_c) {
        if (masked) launch(count, wide_c, std::true_type{});
        else launch(count, wide_c, std::false_type{});
    };
    auto with_wide = [&](auto count) {
        if (wide) with_masked(count, std::true_type{});
        else with_masked(count, std::false_type{});
    };
    if (c.count) with_wide(std::true_type{});
    else with_wide(std::false_type{});
    LAUNCH_CHECK("k_raster");
    return SD7_OK;
}

sd7_status do_raster_bwd(const Call& c)
{
    const sd7_layout& L = c.P.L;
    sd7_status s = fill(c, c.at<uint32_t>(L.off_d_splat), 9 * (size_t)L.n_total, 0);
    if (s != SD7_OK) return s;
    k_raster_bwd<<<c.P.tblocks, 64, 0, c.st>>>(c.tab, c.P.tmap, c.at<uint2>(L.off_ranges),
                                                 c.at<uint32_t>(L.off_pair_g), c.at<float4>(L.off_splat),
                                                 c.at<float>(L.off_d_splat));
    LAUNCH_CHECK("k_raster_bwd");
    return SD7_OK;
}

sd7_status do_project_bwd(const Call& c)
{
    const sd7_layout& L = c.P.L;
    if (c.P.gblocks == 0) return SD7_OK;
    k_project_bwd<<<c.P.gblocks, kBlock, 0, c.st>>>(c.tab, c.P.gmap, c.at<float>(L.off_mu_c), c.at<float>(L.off_cov_c),
                                                     c.at<float>(L.off_alpha_c), c.at<uint32_t>(L.off_depth_key),
                                                     c.at<float>(L.off_d_splat), c.at<float>(L.off_d_mu_c),
                                                     c.at<float>(L.off_d_cov_c), c.at<float>(L.off_d_alpha_c));
    LAUNCH_CHECK("k_project_bwd");
    return SD7_OK;
}

sd7_status do_slice_bwd(const Call& c, const sd7_frame* frames, int nf)
{
    const sd7_layout& L = c.P.L;
    if (c.P.gblocks == 0) return SD7_OK;
    for (int a = 0; a < nf; ++a)
        for (int b = a + 1; b < nf; ++b)
            if (frames[a].scene.n > 0 && frames[a].grad.L == frames[b].grad.L)
                return fail(SD7_EINVAL, "frames %d and %d share gradient buffers", a, b);
    k_slice_bwd<<<c.P.gblocks, kBlock, 0, c.st>>>(c.tab, c.P.gmap, c.at<float>(L.off_d_mu_c),
                                                   c.at<float>(L.off_d_cov_c), c.at<float>(L.off_d_alpha_c));
    LAUNCH_CHECK("k_slice_bwd");
    return SD7_OK;
}

}  // namespace

extern "C" {

const char* sd7_last_error(void) { return g_err; }

sd7_status sd7_create(int device, sd7_ctx** out)
{
    g_err[0] = 0;
    if (!out) return fail(SD7_EINVAL, "out is NULL");
    *out = nullptr;
    int count = 0;
    HIP_TRY(hipGetDeviceCount(&count));
    if (device < 0 || device >= count) return fail(SD7_EINVAL, "device %d outside [0, %d)", device, count);
    HIP_TRY(hipSetDevice(device));
    // k_tile_count keeps one counter per tile of a frame in LDS (up to 128 KB)
    HIP_TRY(hipFuncSetAttribute(reinterpret_cast<const void*>(&k_tile_count),
                                hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)(sizeof(uint32_t) * kMaxCountTiles)));
    void* sp = nullptr;
    HIP_TRY(hipGetSymbolAddress(&sp, HIP_SYMBOL(scratch)));
    if (!sp) return fail(SD7_EHIP, "hipGetSymbolAddress gave no address for the static workspace");
    sd7_ctx* c = new (std::nothrow) sd7_ctx();
    if (!c) return fail(SD7_ENOMEM, "out of host memory");
    c->device = device;
    c->scratch = static_cast<char*>(sp);
    c->slot_bytes = align_up(sizeof(FrameDev) * SD7_MAX_FRAMES);
    hipError_t e = hipHostMalloc((void**)&c->ring, c->slot_bytes * kRing, hipHostMallocDefault);
    if (e != hipSuccess) {
        delete c;
        return fail(SD7_EHIP, "hipHostMalloc: %s", hipGetErrorString(e));
    }
    for (int i = 0; i < kRing; ++i) {
        c->used[i] = false;
        e = hipEventCreateWithFlags(&c->ev[i], hipEventDisableTiming);
        if (e != hipSuccess) {
            for (int j = 0; j < i; ++j) (void)hipEventDestroy(c->ev[j]);
            (void)hipHostFree(c->ring);
            delete c;
            return fail(SD7_EHIP, "hipEventCreate: %s", hipGetErrorString(e));
        }
    }
    const char* pf = std::getenv("SD7_PROFILE");
    if (pf && pf[0] && std::strcmp(pf, "0") != 0) {
        int made = 0;
        for (; made < kProfSlots; ++made) {
            if (hipEventCreate(&c->pf_start[made]) != hipSuccess) break;
            if (hipEventCreate(&c->pf_end[made]) != hipSuccess) {
                (void)hipEventDestroy(c->pf_start[made]);
                break;
            }
        }
        if (made < kProfSlots) {
            for (int j = 0; j < made; ++j) {
                (void)hipEventDestroy(c->pf_start[j]);
                (void)hipEventDestroy(c->pf_end[j]);
            }
            for (int i = 0; i < kRing; ++i) (void)hipEventDestroy(c->ev[i]);
            (void)hipHostFree(c->ring);
            delete c;
            return fail(SD7_EHIP, "hipEventCreate for SD7_PROFILE failed");
        }
        c->profile = true;
    }
    *out = c;
    return SD7_OK;
}

sd7_status sd7_profile_read(sd7_ctx* ctx, sd7_stage_time* out, int max, int* count, int reset)
{
    g_err[0] = 0;
    if (!ctx || !count || (max > 0 && !out) || max < 0) return fail(SD7_EINVAL, "ctx/count/out invalid");
    *count = 0;
    if (!ctx->profile) return SD7_OK;
    HIP_TRY(hipSetDevice(ctx->device));
    std::lock_guard<std::mutex> lock(ctx->pf_mu);
    while (ctx->pf_n > 0) {
        const sd7_status s = profile_retire(ctx);
        if (s != SD7_OK) return s;
    }
    int n = 0;
    for (int st = 0; st < kPStages; ++st) {
        if (ctx->pf_calls[st] == 0) continue;
        if (n < max) out[n] = sd7_stage_time{kProfNames[st], ctx->pf_calls[st], ctx->pf_total[st], ctx->pf_max[st]};
        ++n;
    }
    *count = std::min(n, max);
    if (reset) {
        for (int st = 0; st < kPStages; ++st) {
            ctx->pf_calls[st] = 0;
            ctx->pf_total[st] = ctx->pf_max[st] = 0.0;
        }
    }
    return SD7_OK;
}

void sd7_destroy(sd7_ctx* ctx)
{
    if (!ctx) return;
    (void)hipSetDevice(ctx->device);
    for (int i = 0; i < kRing; ++i) {
        if (ctx->used[i]) (void)hipEventSynchronize(ctx->ev[i]);
        (void)hipEventDestroy(ctx->ev[i]);
    }
    if (ctx->profile) {
        (void)hipDeviceSynchronize();
        for (int k = 0; k < kProfSlots; ++k) {
            (void)hipEventDestroy(ctx->pf_start[k]);
            (void)hipEventDestroy(ctx->pf_end[k]);
        }
    }
    (void)hipHostFree(ctx->ring);
    delete ctx;
}

sd7_status sd7_plan(const sd7_frame* frames, int nf, int64_t pair_capacity, sd7_layout* out)
{
    g_err[0] = 0;
    if (!out) return fail(SD7_EINVAL, "out is NULL");
    Plan P;
    sd7_status s = make_plan(frames, nf, pair_capacity, P, false);
    if (s == SD7_OK) *out = P.L;
    return s;
}

#define STAGE(name, bwd, ...)                                                                        \
    sd7_status name(sd7_ctx* ctx, const sd7_frame* frames, int nf, int64_t cap, void* ws, size_t ws_bytes, \
                    sd7_stream stream)                                                                \
    {                                                                                                 \
        Call c;                                                                                       \
        sd7_status s = begin(ctx, frames, nf, cap, ws, ws_bytes, stream, c, bwd);                     \
        if (s != SD7_OK) return s;                                                                    \
        __VA_ARGS__                                                                                   \
    }

STAGE(sd7_slice, false, { return timed(c, kPSlice, [&] { return do_slice(c); }); })
STAGE(sd7_project, false, { return timed(c, kPProject, [&] { return do_project(c); }); })
STAGE(sd7_slice_project, false, { return timed(c, kPSliceProject, [&] { return do_slice_project(c); }); })
STAGE(sd7_bin, false, { return timed(c, kPBin, [&] { return do_bin(c); }); })
STAGE(sd7_rasterize, false, { return timed(c, kPRaster, [&] { return do_raster(c); }); })
STAGE(sd7_render, false, {
    if ((s = timed(c, kPSliceProject, [&] { return do_slice_project(c); })) != SD7_OK) return s;
    if ((s = timed(c, kPBin, [&] { return do_bin(c); })) != SD7_OK) return s;
    return timed(c, kPRaster, [&] { return do_raster(c); });
})
STAGE(sd7_rasterize_backward, true, { return timed(c, kPRasterBwd, [&] { return do_raster_bwd(c); }); })

}  // extern "C"

struct sd7_graph {
    sd7_ctx* ctx = nullptr;
    Plan P;
    char* ws = nullptr;
    int nf = 0;
    int64_t cap = 0;
    bool count = false, agr = false;
    int64_t n[SD7_MAX_FRAMES];
    int32_t W[SD7_MAX_FRAMES], H[SD7_MAX_FRAMES];
    bool has_count[SD7_MAX_FRAMES], has_agr[SD7_MAX_FRAMES];
    int same_as[SD7_MAX_FRAMES];  // first frame with the same scene arrays
    hipGraphExec_t exec = nullptr;
};

// For each frame, the first frame of the call with the same scene (the same
// six parameter arrays and n): the grouping the fused slice/projection's
// launch is planned on.
void scene_sharing(const sd7_frame* fr, int nf, int* same_as)
{
    for (int f = 0; f < nf; ++f) {
        same_as[f] = f;
        const sd7_scene& A = fr[f].scene;
        for (int h = 0; h < f; ++h) {
            const sd7_scene& B = fr[h].scene;
            if (A.n == B.n && A.mu_p == B.mu_p && A.mu_t == B.mu_t && A.mu_d == B.mu_d && A.L == B.L &&
                A.alpha == B.alpha && A.sh == B.sh) {
                same_as[f] = h;
                break;
            }
        }
    }
}

extern "C" {

sd7_status sd7_graph_create(sd7_ctx* ctx, const sd7_frame* frames, int nf, int64_t cap, void* ws, size_t ws_bytes,
                            sd7_graph** out)
{
    g_err[0] = 0;
    if (!out) return fail(SD7_EINVAL, "out is NULL");
    *out = nullptr;
    Call c;
    sd7_status s = prepare(ctx, frames, nf, cap, ws, ws_bytes, nullptr, c, false);
    if (s != SD7_OK) return s;
    sd7_graph* g = new (std::nothrow) sd7_graph();
    if (!g) return fail(SD7_ENOMEM, "out of host memory");
    g->ctx = ctx;
    g->P = c.P;
    g->ws = c.ws;
    g->nf = nf;
    g->cap = cap;
    g->count = c.count;
    g->agr = c.agr;
    for (int f = 0; f < nf; ++f) {
        g->n[f] = frames[f].scene.n;
        g->W[f] = frames[f].view.W;
        g->H[f] = frames[f].view.H;
        g->has_count[f] = frames[f].ncontrib != nullptr;
        g->has_agr[f] = frames[f].scene.agr != nullptr;
    }
    scene_sharing(frames, nf, g->same_as);
    // capture the render's launches (kernels only: the clears are fill
    // kernels) on a private stream of default priority
    hipStream_t st = nullptr;
    hipError_t e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
    if (e != hipSuccess) {
        delete g;
        return fail(SD7_EHIP, "hipStreamCreateWithFlags: %s", hipGetErrorString(e));
    }
    c.st = st;
    hipGraph_t graph = nullptr;
    e = hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
        s = do_slice_project(c);
        if (s == SD7_OK) s = do_bin(c);
        if (s == SD7_OK) s = do_raster(c);
        const hipError_t e2 = hipStreamEndCapture(st, &graph);
        if (s == SD7_OK && e2 != hipSuccess) s = fail(SD7_EHIP, "hipStreamEndCapture: %s", hipGetErrorString(e2));
    } else {
        s = fail(SD7_EHIP, "hipStreamBeginCapture: %s", hipGetErrorString(e));
    }
    if (s == SD7_OK) {
        e = hipGraphInstantiate(&g->exec, graph, nullptr, nullptr, 0);
        if (e != hipSuccess) s = fail(SD7_EHIP, "hipGraphInstantiate: %s", hipGetErrorString(e));
    }
    if (graph) (void)hipGraphDestroy(graph);
    (void)hipStreamDestroy(st);
    if (s != SD7_OK) {
        delete g;
        return s;
    }
    *out = g;
    return SD7_OK;
}

sd7_status sd7_graph_launch(sd7_graph* g, const sd7_frame* frames, int nf, sd7_stream stream)
{
    g_err[0] = 0;
    if (!g || !frames) return fail(SD7_EINVAL, "graph or frames is NULL");
    if (nf != g->nf) return fail(SD7_EINVAL, "nf=%d, the graph was captured for %d frames", nf, g->nf);
    int same_as[SD7_MAX_FRAMES];
    scene_sharing(frames, nf, same_as);
    for (int f = 0; f < nf; ++f) {
        if (same_as[f] != g->same_as[f])
            return fail(SD7_EINVAL, "frame %d: frames share scenes differently from the captured frames", f);
        const sd7_frame& F = frames[f];
        if (F.scene.n != g->n[f] || F.view.W != g->W[f] || F.view.H != g->H[f] ||
            (F.ncontrib != nullptr) != g->has_count[f] || (F.scene.agr != nullptr) != g->has_agr[f])
            return fail(SD7_EINVAL, "frame %d: Gaussian count, resolution, contributor counts or AGR differ "
                        "from the captured frame", f);
        if (F.scene.n > 0 && (!F.scene.mu_p || !F.scene.mu_t || !F.scene.mu_d || !F.scene.L || !F.scene.alpha ||
                              !F.scene.sh))
            return fail(SD7_EINVAL, "frame %d: NULL scene array", f);
        if (!F.image || !F.final_T || !F.last) return fail(SD7_EINVAL, "frame %d: NULL image/final_T/last", f);
        if (!(F.view.fx > 0.f) || !(F.view.fy > 0.f)) return fail(SD7_EINVAL, "frame %d: focal length must be > 0", f);
    }
    HIP_TRY(hipSetDevice(g->ctx->device));
    hipStream_t st = static_cast<hipStream_t>(stream);
    sd7_status s = upload_table(g->ctx, frames, nf, g->P, g->ws, st);
    if (s != SD7_OK) return s;
    HIP_TRY(hipGraphLaunch(g->exec, st));
    return SD7_OK;
}

void sd7_graph_destroy(sd7_graph* g)
{
    if (!g) return;
    (void)hipSetDevice(g->ctx->device);
    if (g->exec) (void)hipGraphExecDestroy(g->exec);
    delete g;
}

sd7_status sd7_render_static(sd7_ctx* ctx, const sd7_frame* frames, int nf, int64_t cap, uint32_t* counts_out,
                             sd7_stream stream)
{
    g_err[0] = 0;
    if (!ctx) return fail(SD7_EINVAL, "ctx is NULL");
    Call c;
    sd7_status s = make_plan(frames, nf, cap, c.P, false);
    if (s != SD7_OK) return s;
    if (c.P.L.bytes > (size_t)SD7_STATIC_WS_BYTES)
        return fail(SD7_EWORKSPACE, "these frames need a %zu-byte workspace; the static one holds %zu",
                    c.P.L.bytes, (size_t)SD7_STATIC_WS_BYTES);
    s = begin(ctx, frames, nf, cap, ctx->scratch, SD7_STATIC_WS_BYTES, stream, c, false);
    if (s != SD7_OK) return s;
    if ((s = timed(c, kPSliceProject, [&] { return do_slice_project(c); })) != SD7_OK) return s;
    if ((s = timed(c, kPBin, [&] { return do_bin(c); })) != SD7_OK) return s;
    if ((s = timed(c, kPRaster, [&] { return do_raster(c); })) != SD7_OK) return s;
    if (counts_out) {
        k_copy_u32<<<1, 256, 0, c.st>>>(counts_out, c.counts, (uint32_t)(SD7_CNT_WORDS * nf));
        LAUNCH_CHECK("k_copy_u32");
    }
    return SD7_OK;
}
STAGE(sd7_project_backward, true, { return timed(c, kPProjectBwd, [&] { return do_project_bwd(c); }); })
STAGE(sd7_slice_backward, true, { return timed(c, kPSliceBwd, [&] { return do_slice_bwd(c, frames, nf); }); })

sd7_status sd7_cov_decompose(sd7_ctx* ctx, int64_t n, const float* cov, float* scale, float* rot,
                             sd7_stream stream)
{
    g_err[0] = 0;
    if (!ctx) return fail(SD7_EINVAL, "ctx is NULL");
    if (n < 0 || n >= (int64_t)1 << 31) return fail(SD7_EINVAL, "n=%lld outside [0, 2^31)", (long long)n);
    if (n == 0) return SD7_OK;
    if (!cov || !scale || !rot) return fail(SD7_EINVAL, "NULL array");
    HIP_TRY(hipSetDevice(ctx->device));
    k_cov_decompose<<<ceil_div(n, kBlock), kBlock, 0, static_cast<hipStream_t>(stream)>>>((uint32_t)n, cov, scale,
                                                                                          rot);
    LAUNCH_CHECK("k_cov_decompose");
    return SD7_OK;
}

sd7_status sd7_split_test(sd7_ctx* ctx, const sd7_scene* scene, float extent, float time_span, uint8_t* out,
                          sd7_stream stream)
{
    g_err[0] = 0;
    if (!ctx || !scene) return fail(SD7_EINVAL, "ctx or scene is NULL");
    const int64_t n = scene->n;
    if (n < 0 || n >= (int64_t)1 << 31) return fail(SD7_EINVAL, "n=%lld outside [0, 2^31)", (long long)n);
    if (!(extent > 0.f) || !(time_span > 0.f)) return fail(SD7_EINVAL, "extent and time_span must be > 0");
    if (n == 0) return SD7_OK;
    if (!scene->L || !out) return fail(SD7_EINVAL, "NULL array");
    HIP_TRY(hipSetDevice(ctx->device));
    k_split_test<<<ceil_div(n, kBlock), kBlock, 0, static_cast<hipStream_t>(stream)>>>((uint32_t)n, scene->L,
                                                                                       extent, time_span, out);
    LAUNCH_CHECK("k_split_test");
    return SD7_OK;
}

sd7_status sd7_adam_step(sd7_ctx* ctx, int64_t n, const sd7_arrays* params, const sd7_scene_grad* grad,
                         const sd7_arrays* m, const sd7_arrays* v, const sd7_adam* cfg, sd7_stream stream)
{
    g_err[0] = 0;
    if (!ctx || !params || !grad || !m || !v || !cfg) return fail(SD7_EINVAL, "NULL argument");
    if (n < 0 || n >= (int64_t)1 << 31) return fail(SD7_EINVAL, "n=%lld outside [0, 2^31)", (long long)n);
    if (cfg->step < 1) return fail(SD7_EINVAL, "step=%d must be >= 1", cfg->step);
    if (!(cfg->beta1 >= 0.f && cfg->beta1 < 1.f && cfg->beta2 >= 0.f && cfg->beta2 < 1.f && cfg->eps > 0.f))
        return fail(SD7_EINVAL, "need 0 <= beta1, beta2 < 1 and eps > 0");
    if (n == 0) return SD7_OK;
    ArraySet P, G, M, V;
    const float* gp[6] = {grad->mu_p, grad->mu_t, grad->mu_d, grad->L, grad->alpha, grad->sh};
    float* pp[6] = {params->mu_p, params->mu_t, params->mu_d, params->L, params->alpha, params->sh};
    float* mp[6] = {m->mu_p, m->mu_t, m->mu_d, m->L, m->alpha, m->sh};
    float* vp[6] = {v->mu_p, v->mu_t, v->mu_d, v->L, v->alpha, v->sh};
    for (int k = 0; k < 6; ++k) {
        if (!gp[k] || !pp[k] || !mp[k] || !vp[k]) return fail(SD7_EINVAL, "NULL array in group %d", k);
        P.a[k] = pp[k]; G.a[k] = const_cast<float*>(gp[k]); M.a[k] = mp[k]; V.a[k] = vp[k];
    }
    AdamArgs a;
    for (int k = 0; k < 6; ++k) a.lr[k] = cfg->lr[k];
    a.beta1 = cfg->beta1; a.beta2 = cfg->beta2; a.eps = cfg->eps;
    a.rbc1 = (float)(1.0 / (1.0 - std::pow((double)cfg->beta1, cfg->step)));
    a.rsbc2 = (float)(1.0 / std::sqrt(1.0 - std::pow((double)cfg->beta2, cfg->step)));
    a.alpha_lo = cfg->alpha_lo; a.alpha_hi = cfg->alpha_hi; a.diag_min = cfg->diag_min;
    HIP_TRY(hipSetDevice(ctx->device));
    const uint32_t chunks = ceil_div((uint64_t)n, (uint64_t)kBlock * kAdamPerThread);
    k_adam<<<84u * chunks, kBlock, 0, static_cast<hipStream_t>(stream)>>>((uint32_t)n, chunks, P, G, M, V, a);
    LAUNCH_CHECK("k_adam");
    return SD7_OK;
}

size_t sd7_prune_workspace_size(int64_t n)
{
    return n < 0 ? 0 : prune_ws(n).bytes;
}

sd7_status sd7_prune_count(sd7_ctx* ctx, int64_t n, const float* alpha, float tau, void* ws, size_t ws_bytes,
                           uint32_t* d_kept, sd7_stream stream)
{
    g_err[0] = 0;
    if (!ctx || !d_kept || !ws) return fail(SD7_EINVAL, "NULL argument");
    if (n < 0 || n >= (int64_t)1 << 31) return fail(SD7_EINVAL, "n=%lld outside [0, 2^31)", (long long)n);
    const PruneWs w = prune_ws(n);
    if (ws_bytes < w.bytes) return fail(SD7_EWORKSPACE, "workspace has %zu bytes, %zu needed", ws_bytes, w.bytes);
    if (reinterpret_cast<uintptr_t>(ws) % kAlign) return fail(SD7_EINVAL, "workspace not 256-byte aligned");
    if (n > 0 && !alpha) return fail(SD7_EINVAL, "alpha is NULL");
    HIP_TRY(hipSetDevice(ctx->device));
    hipStream_t st = static_cast<hipStream_t>(stream);
    char* base = static_cast<char*>(ws);
    uint32_t* keep = reinterpret_cast<uint32_t*>(base + w.keep);
    uint32_t* pos = reinterpret_cast<uint32_t*>(base + w.pos);
    if (n == 0) {
        k_prune_total<<<1, 64, 0, st>>>(0, keep, pos, d_kept);
        LAUNCH_CHECK("k_prune_total");
        return SD7_OK;
    }
    k_prune_flags<<<ceil_div(n, kBlock), kBlock, 0, st>>>((uint32_t)n, alpha, tau, keep, pos);
    LAUNCH_CHECK("k_prune_flags");
    sd7_status s = scan_with(st, reinterpret_cast<uint32_t*>(base + w.part), pos, (uint32_t)n, nullptr,
                             (uint32_t)n, nullptr);
    if (s != SD7_OK) return s;
    k_prune_total<<<1, 64, 0, st>>>((uint32_t)n, keep, pos, d_kept);
    LAUNCH_CHECK("k_prune_total");
    return SD7_OK;
}

sd7_status sd7_prune_apply(sd7_ctx* ctx, int64_t n, int64_t n_kept, const float* const* src, float* const* dst,
                           const int32_t* planes, int narrays, const void* ws, size_t ws_bytes, sd7_stream stream)
{
    g_err[0] = 0;
    if (!ctx || !ws || (narrays > 0 && (!src || !dst || !planes))) return fail(SD7_EINVAL, "NULL argument");
    if (n < 0 || n >= (int64_t)1 << 31 || n_kept < 0 || n_kept > n)
        return fail(SD7_EINVAL, "need 0 <= n_kept <= n < 2^31");
    if (narrays < 0 || narrays > kMaxPruneArrays) return fail(SD7_EINVAL, "narrays=%d outside [0, %d]", narrays,
                                                              kMaxPruneArrays);
    const PruneWs w = prune_ws(n);
    if (ws_bytes < w.bytes) return fail(SD7_EWORKSPACE, "workspace has %zu bytes, %zu needed", ws_bytes, w.bytes);
    if (n == 0 || n_kept == 0) return SD7_OK;  // nothing to copy (arrays may be empty)
    PruneArrays pa;
    std::memset(&pa, 0, sizeof(pa));
    pa.narrays = narrays;
    uint64_t tot = 0;
    for (int j = 0; j < narrays; ++j) {
        if (!src[j] || !dst[j] || planes[j] < 1) return fail(SD7_EINVAL, "array %d: NULL or planes < 1", j);
        pa.src[j] = src[j];
        pa.dst[j] = dst[j];
        pa.plane0[j] = (uint32_t)tot;
        tot += (uint64_t)planes[j];
    }
    pa.plane0[narrays] = (uint32_t)tot;
    if (tot == 0) return SD7_OK;
    HIP_TRY(hipSetDevice(ctx->device));
    const char* base = static_cast<const char*>(ws);
    const uint32_t chunks = ceil_div(n, kBlock);
    if (tot * chunks >= (1ull << 31)) return fail(SD7_EINVAL, "too many planes x Gaussians");
    k_prune_apply<<<(uint32_t)(tot * chunks), kBlock, 0, static_cast<hipStream_t>(stream)>>>(
        (uint32_t)n, (uint32_t)n_kept, chunks, reinterpret_cast<const uint32_t*>(base + w.keep),
        reinterpret_cast<const uint32_t*>(base + w.pos), pa);
    LAUNCH_CHECK("k_prune_apply");
    return SD7_OK;
}

sd7_status sd7_read_counts(sd7_ctx* ctx, int nf, const void* ws, uint32_t* out, sd7_stream stream)
{
    g_err[0] = 0;
    if (!ctx || !ws || !out) return fail(SD7_EINVAL, "NULL argument");
    if (nf < 1 || nf > SD7_MAX_FRAMES) return fail(SD7_EINVAL, "nf=%d outside [1, %d]", nf, SD7_MAX_FRAMES);
    HIP_TRY(hipSetDevice(ctx->device));
    const size_t off = align_up(sizeof(FrameDev) * nf);
    HIP_TRY(hipStreamSynchronize(static_cast<hipStream_t>(stream)));
    HIP_TRY(hipMemcpy(out, static_cast<const char*>(ws) + off, sizeof(uint32_t) * SD7_CNT_WORDS * nf,
                      hipMemcpyDeviceToHost));
    return SD7_OK;
}

}  // extern "C"
