// cm_batch.hip -- the tiled (owner-computes) path for one or many windows.
//
// Scattered global floating-point atomics run at about 22 G/s on MI355X
// whatever the array size (one request per distinct cache line), while LDS
// FP64 atomics run at about 1.4 T/s.  So instead of splatting every tap with a
// global atomic, each warped position becomes a record binned by the 32x32
// tile of its tap (x0, y0) (a counting sort: count, scan, scatter), and one
// workgroup per tile accumulates its records in LDS and writes the pixels it
// owns that some tap reached, once, with plain stores.  A record's taps can
// reach one column right of and one row below its tile; that halo goes to a
// small buffer and a merge pass adds it, in a fixed order, into column 0 /
// row 0 of the neighbouring tiles.
//
// Forward:  count -> chunk sums -> chunk scan -> scan -> offsets -> scatter
//           -> tile -> merge -> finalize.  The count also stores each event's
//           mask, so the scatter warps valid events only.  The per-reference
//           sums of Eq. 1 are reduced in the tile (interior) and merge
//           (border) kernels.
// Backward: the same sort over flow-sampling positions; the sweep re-runs
//           each event's warp, gathers the adjoint seeds, runs the reverse
//           sweep and emits one record per sampling position with
//           dt * adjoint; the tile kernels turn the accumulated dL/du into
//           d rho and d theta per pixel.
//
// Every kernel covers all windows of a batch in one launch: per-window
// metadata (WinMeta) lives in device memory, and a table kernel run first in
// each call finds the window of every event block, bin and tile (binary search
// over prefix offsets), the motion coefficients of every flow set and, per
// forward bin, the few values its tile and merge kernels need.  A single
// window is a batch of one.
#include <type_traits>

#include "cm_kernels.hpp"

namespace cm {

// ---------------------------------------------------------------------------
// Window lookup
// ---------------------------------------------------------------------------

// Largest w with key >= field(meta[w]) (fields are nondecreasing in w).
template <typename F>
__device__ __forceinline__ int find_window(const WinMeta* __restrict__ meta, int nw, int64_t key,
                                           F field)
{
    int lo = 0, hi = nw - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (field(meta[mid]) <= key) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

__device__ __forceinline__ int window_of_block(const WinMeta* meta, int nw, int64_t b)
{
    return find_window(meta, nw, b, [](const WinMeta& m) { return m.blk_off; });
}

// Workgroups go to the XCDs round-robin (workgroup b runs on XCD b % 8), and
// each XCD has its own L2.  The event-block kernels renumber their workgroups
// so that every XCD takes one contiguous range of event blocks: the blocks of
// a window then gather its inverse depth and splat images through one L2
// instead of all eight fetching the same lines.  A bijection of [0, n).
constexpr uint32_t kXcds = 8;

__device__ __forceinline__ int64_t xcd_block()
{
    const uint32_t b = blockIdx.x, n = gridDim.x;
    const uint32_t q = n / kXcds, r = n % kXcds, x = b % kXcds, i = b / kXcds;
    return (int64_t)x * q + min(x, r) + i;
}

// One lane's next event, loaded an iteration ahead so that its latency
// overlaps the current event's warp and gathers.
struct EventPrefetch {
    struct Ev {
        float x, y, t;
        int8_t p;
    };
    const float* __restrict__ ex;
    const float* __restrict__ ey;
    const float* __restrict__ et;
    const int8_t* __restrict__ ep;
    int64_t n;
    Ev nxt;
    __device__ __forceinline__ EventPrefetch(const float* x, const float* y, const float* t,
                                             const int8_t* p, int64_t k, int64_t n_)
        : ex(x), ey(y), et(t), ep(p), n(n_)
    {
        load(k);
    }
    __device__ __forceinline__ void load(int64_t k)
    {
        if (k < n) {
            nxt.x = ex[k];
            nxt.y = ey[k];
            nxt.t = et[k];
            nxt.p = ep ? ep[k] : (int8_t)0;
        }
    }
    // The event loaded last; starts loading event k (k >= n: nothing).
    __device__ __forceinline__ Ev take(int64_t k)
    {
        const Ev cur = nxt;
        load(k);
        return cur;
    }
};

// ---------------------------------------------------------------------------
// Deterministic mode helpers (one wavefront per block)
// ---------------------------------------------------------------------------

__device__ __forceinline__ uint64_t lanes_below()
{
    return (1ull << __lane_id()) - 1ull;
}

// Slot of this lane's record in bin `bin`: counter[bin] plus the number of
// active lanes with the same bin and a lower lane id; the counter then advances
// by the group's size.  Lanes are served in lane order, so, with one wavefront
// per block, a block's records land in each bin in (event, step) order.
__device__ __forceinline__ uint32_t stable_slot(uint32_t* counter, int bin)
{
    uint64_t todo = __ballot(1);
    uint32_t slot = 0;
    while (todo) {
        const int leader = __ffsll((unsigned long long)todo) - 1;
        const int b = __shfl(bin, leader);
        const uint64_t same = __ballot(bin == b);
        const uint32_t base = counter[b];
        if (bin == b) slot = base + (uint32_t)__popcll(same & lanes_below());
        if ((int)__lane_id() == leader) counter[b] = base + (uint32_t)__popcll(same);
        todo &= ~same;
    }
    return slot;
}

// Adds (vx, vy) of every lane with `act` into cell[key], lanes with equal keys
// in lane order, each add applied to the running value: the canonical order
// of the deterministic mode.  Called by all lanes of the wavefront.
__device__ __forceinline__ void ordered_add(double2* cells, bool act, int key, double vx, double vy)
{
    uint64_t todo = __ballot(act);
    while (todo) {
        const int leader = __ffsll((unsigned long long)todo) - 1;
        const int k = __shfl(key, leader);
        const uint64_t same = __ballot(act && key == k);
        double2 v = cells[k];
        uint64_t m = same;
        while (m) {
            const int l = __ffsll((unsigned long long)m) - 1;
            v.x += __shfl(vx, l);
            v.y += __shfl(vy, l);
            m &= m - 1;
        }
        if ((int)__lane_id() == leader) cells[k] = v;
        todo &= ~same;
    }
}

// ---------------------------------------------------------------------------
// Counting sort of records into bins
// ---------------------------------------------------------------------------

// Fills the block's table of reference times (and, with hdr, the adjoint
// seed coefficients) for window P.
__device__ __forceinline__ void load_ref_table(const WinParams& P, const StateHeader* hdr,
                                               RefTable& rt)
{
    if (threadIdx.x < kMaxRefs) {
        const int r = threadIdx.x;
        rt.t[r] = P.refs[r];
        rt.coef[r] = (hdr && r < P.R) ? P.two_over_R / (hdr->nact[r] + P.eps) : 0.0;
        rt.sf[r] = P.sf[r];
        rt.sb[r] = P.sb[r];
    }
}

// The count and sweep kernels ask for 3 waves per SIMD: their 16-reference
// instances would otherwise need 170-180 VGPRs and run 2 waves; the few
// spilled registers cost less than the lost latency hiding (the scatter,
// which holds every visit's position until its records are written, loses
// more to spills and is left at 2).
//
// Atomic mode (DET false): every tile owns all its pixels, so a position is
// counted in each tile its taps reach (tiles_reached), and each valid event
// once more in a source bin: the tile of its own position (with the tiles its
// taps reach) when the batch's backward samples the flow at the events only
// (`ae`), else the tile of its reference-0 position.  A block reserves its
// range in every bin it fills with one returning atomic on the bin's total,
// and stores the offset it got in its histogram row.  Deterministic mode:
// reference bins only, the row holds counts, and the chunk sums feed the
// column scan that orders the blocks.
template <int RM, int NT, int FM, bool DET>
__global__ __launch_bounds__(NT, 3) void fwd_count_kernel(
    const WinMeta* __restrict__ meta, int nw, const int* __restrict__ win_of, const float* __restrict__ ex,
    const float* __restrict__ ey, const float* __restrict__ et, const float* __restrict__ rho,
    const float* __restrict__ ego, const Motion* __restrict__ mtab, uint32_t* __restrict__ hist,
    uint32_t* __restrict__ csum, uint32_t* __restrict__ totals, uint32_t* __restrict__ totals_src,
    int ae, StateHeader* __restrict__ hdrs, uint8_t* __restrict__ valid)
{
    extern __shared__ uint32_t lh[];
    __shared__ uint32_t cnt_lds;
    __shared__ uint32_t bins[RM][NT];
    const int64_t blk = xcd_block();
    const int w = win_of[blk];
    const WinParams& P = meta[w].P;
    const TileGeom G = meta[w].G;
    const int64_t lb = blk - meta[w].blk_off;
    const int64_t ev0 = meta[w].ev_off, n = meta[w].n;
    const int nrb = G.nbins;                    // reference bins; source bins follow
    const int nlb = DET ? nrb : nrb + G.nbins_s;
    __shared__ RefTable rt;
    for (int i = threadIdx.x; i < nlb; i += blockDim.x) lh[i] = 0;
    if (threadIdx.x == 0) cnt_lds = 0;
    load_ref_table(P, nullptr, rt);
    __shared__ MotionTable mt;
    const Flows<FM> u = make_flows_tab<FM>(P, rho + meta[w].pix_off, ego + 6 * meta[w].ego_off,
                                           mtab + meta[w].ego_off, &mt);
    __syncthreads();
    const int64_t base = lb * NT * G.ept;
    uint32_t cnt = 0;
    // the next iteration's event is loaded before this one is warped
    EventPrefetch nx(ex + ev0, ey + ev0, et + ev0, nullptr, base + threadIdx.x, n);
    for (int e = 0; e < G.ept; ++e) {
        const int64_t k = base + (int64_t)e * NT + threadIdx.x;
        if (k >= n) break;
        const EventPrefetch::Ev cur = nx.take(e + 1 < G.ept ? k + NT : n);
        // only the bins are kept, in the thread's LDS column (registers
        // would stay live through the whole warp)
        Visits v;
        uint32_t t0 = 0;        // tile of the reference-0 position
        const bool ok = warp_visits_v<RM, FM>(P, u, rt, cur.x, cur.y, cur.t, v,
                                              [&](int j, double X, double Y, int r) {
                                                  const Taps tp = make_taps(P, X, Y);
                                                  if (DET) {
                                                      bins[j][threadIdx.x] =
                                                          r * G.ntiles + tile_index(G, tp);
                                                  } else {
                                                      const uint32_t tr = tiles_reached(G, tp);
                                                      bins[j][threadIdx.x] =
                                                          tr + (uint32_t)(r * G.ntiles);
                                                      if (r == 0) t0 = tr & 0xffffu;
                                                  }
                                              });
        // the mask, for the scatter (which then warps valid events only)
        valid[ev0 + k] = ok ? 1 : 0;
        if (!ok) continue;
        ++cnt;
#pragma unroll
        for (int j = 0; j < RM; ++j) {
            if (j < P.R) {
                if (DET) atomicAdd(&lh[bins[j][threadIdx.x]], 1u);
                else for_each_reached(bins[j][threadIdx.x], G.ntx,
                                      [&](int b) { atomicAdd(&lh[b], 1u); });
            }
        }
        if (!DET) {
            if (ae) for_each_reached(tiles_reached(G, make_taps(P, cur.x, cur.y)), G.ntx,
                                     [&](int t) { atomicAdd(&lh[nrb + t], 1u); });
            else atomicAdd(&lh[nrb + (int)t0], 1u);
        }
    }
    if (cnt) atomicAdd(&cnt_lds, cnt);
    __syncthreads();
    uint32_t* row = hist + meta[w].hist_off + lb * nlb;
    if (DET) {
        uint32_t* cs = csum + meta[w].csum_off + (size_t)(lb / kScanChunk) * G.nbins;
        for (int i = threadIdx.x; i < G.nbins; i += blockDim.x) {
            const uint32_t c = lh[i];
            row[i] = c;
            if (c) atomicAdd(cs + i, c);       // the chunk's column sums (integer: order-free)
        }
    } else {
        for (int i = threadIdx.x; i < nlb; i += blockDim.x) {
            const uint32_t c = lh[i];
            uint32_t* tot = i < nrb ? totals + (meta[w].bin_off + i)
                                    : totals_src + (meta[w].sbin_off + (i - nrb));
            row[i] = c ? atomicAdd(tot, c) : 0u;
        }
    }
    if (threadIdx.x == 0 && cnt_lds) atomicAdd(&hdrs[w].n_valid, (unsigned long long)cnt_lds);
}

// Column scan of each window's block x bin histogram in two levels: blocks
// are grouped in chunks of kScanChunk rows; the count kernels add their rows
// into the chunk sums, then a per-bin scan over chunks, then the per-block
// offsets inside each chunk.  `bwd` selects
// the backward bin space (one bin per flow set and tile).
struct BinSpace {
    __device__ __forceinline__ static int nbins(const WinMeta& m, bool bwd)
    {
        return bwd ? m.G.nbins_b : m.G.nbins;
    }
    __device__ __forceinline__ static int64_t bin_off(const WinMeta& m, bool bwd)
    {
        return bwd ? m.bbin_off : m.bin_off;
    }
    __device__ __forceinline__ static int64_t cell_off(const WinMeta& m, bool bwd)
    {
        return bwd ? m.cell_off_b : m.cell_off_f;
    }
};

// In place: csum[c][bin] <- sum over chunks before c; totals[global bin] = column total.
__global__ __launch_bounds__(256) void chunk_scan_kernel(const WinMeta* __restrict__ meta,
                                                         const int* __restrict__ win_of,
                                                         int64_t nbins_total, int bwd,
                                                         uint32_t* __restrict__ csum,
                                                         uint32_t* __restrict__ totals)
{
    const int64_t gbin = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (gbin >= nbins_total) return;
    const int w = win_of[gbin];
    const WinMeta& M = meta[w];
    const int nbins = BinSpace::nbins(M, bwd);
    const int bin = (int)(gbin - BinSpace::bin_off(M, bwd));
    uint32_t* cs = csum + M.csum_off + bin;
    uint32_t run = 0;
    // eight chunk sums in flight at a time (no serial load-store chain)
    for (int c0 = 0; c0 < M.nchunks; c0 += 8) {
        uint32_t v[8];
#pragma unroll
        for (int i = 0; i < 8; ++i) v[i] = c0 + i < M.nchunks ? cs[(size_t)(c0 + i) * nbins] : 0u;
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            if (c0 + i < M.nchunks) cs[(size_t)(c0 + i) * nbins] = run;
            run += v[i];
        }
    }
    totals[gbin] = run;
}

// Exclusive scan of the bins' totals into start (start[nbins] = the sum), one
// block per bin array (block 0: totals0 -> start0; block 1, if launched:
// totals1 -> start1): chunks of 8192 totals are loaded coalesced into LDS,
// each thread sums 8 consecutive ones, the 1024 sums are scanned with in-wave
// shuffles and the 16 wave totals by one wave, and the results go out
// coalesced.
__global__ __launch_bounds__(1024) void scan_kernel(const uint32_t* __restrict__ totals0,
                                                    int64_t nbins0, uint32_t* __restrict__ start0,
                                                    const uint32_t* __restrict__ totals1,
                                                    int64_t nbins1, uint32_t* __restrict__ start1)
{
    const uint32_t* __restrict__ totals = blockIdx.x ? totals1 : totals0;
    const int64_t nbins = blockIdx.x ? nbins1 : nbins0;
    uint32_t* __restrict__ start = blockIdx.x ? start1 : start0;
    constexpr int T = 1024, K = 8, CH = T * K, NWV = T / 64;
    __shared__ uint32_t buf[CH];
    __shared__ uint32_t wsum[NWV];
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    uint32_t carry = 0;
    for (int64_t base = 0; base < nbins; base += CH) {
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const int64_t i = base + k * T + tid;
            buf[k * T + tid] = i < nbins ? totals[i] : 0u;
        }
        __syncthreads();
        uint32_t v[K], sum = 0;
#pragma unroll
        for (int k = 0; k < K; ++k) {
            v[k] = buf[tid * K + k];
            sum += v[k];
        }
        uint32_t x = sum;                       // inclusive scan within the wave
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const uint32_t y = __shfl_up(x, o, 64);
            if (lane >= o) x += y;
        }
        if (lane == 63) wsum[wid] = x;
        __syncthreads();
        if (wid == 0) {
            uint32_t t = lane < NWV ? wsum[lane] : 0u;
#pragma unroll
            for (int o = 1; o < NWV; o <<= 1) {
                const uint32_t y = __shfl_up(t, o, 64);
                if (lane >= o) t += y;
            }
            if (lane < NWV) wsum[lane] = t;
        }
        __syncthreads();
        uint32_t run = carry + (wid ? wsum[wid - 1] : 0u) + (x - sum);
#pragma unroll
        for (int k = 0; k < K; ++k) {
            buf[tid * K + k] = run;
            run += v[k];
        }
        carry += wsum[NWV - 1];
        __syncthreads();
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const int64_t i = base + k * T + tid;
            if (i < nbins) start[i] = buf[k * T + tid];
        }
        __syncthreads();
    }
    if (tid == 0) start[nbins] = carry;
}

// Atomic mode: the forward's scan, one workgroup per chunk of 8192 bins of
// either array (blocks [0, nc0): the reference bins' chunks, then the source
// bins'): a chunk's first slot is the sum of the totals before it, which its
// workgroup adds up itself (all final when this kernel runs), so the chunks
// scan independently, with no workgroup waiting on another (past
// kScanChunksMax chunks, chunk_sums_kernel first writes each chunk's total,
// and the workgroups add those up instead of the bins before them).
// Each workgroup also lists its chunk's bins, heaviest first: those of at
// least kVeryHeavyBin records, then those of at least kHeavyBin (each class
// in any order), then the rest; the reference list takes the non-empty bins
// (the splat workgroups take it in passes, so the longest bins start first),
// the source list all of them (the order in which a one-workgroup-per-bin
// kernel over them is launched).  A list of capacity cap (the array's bins)
// keeps each class in a region of its own: the rest at [0, cap), the heavy
// bins at [cap, 2 cap), the very heavy ones at [2 cap, 3 cap); its counters,
// cleared by the window table kernel, are the entry count, the very heavy
// and the heavy bins' counts, cap, and the rest's count.  A workgroup
// reserves its entries of each class with one returning atomic.
constexpr uint32_t kHeavyBin = 1024, kVeryHeavyBin = 4096;
constexpr int kListCounters = 8;
constexpr int kScanChunk8k = 8192, kScanChunksMax = 16;

// Entry e of such a list.
__device__ __forceinline__ uint32_t occ_entry(const uint32_t* __restrict__ occ,
                                              const uint32_t* __restrict__ occ_n, uint32_t e)
{
    const uint32_t n2 = occ_n[1], n1 = occ_n[2], cap = occ_n[3];
    if (e < n2) return occ[2 * cap + e];
    if (e < n2 + n1) return occ[cap + (e - n2)];
    return occ[e - n2 - n1];
}

// Each chunk's total (blocks as in scan_chunks_kernel).
__global__ __launch_bounds__(1024) void chunk_sums_kernel(const uint32_t* __restrict__ totals0,
                                                          int64_t nbins0,
                                                          const uint32_t* __restrict__ totals1,
                                                          int64_t nbins1,
                                                          uint32_t* __restrict__ chunk_tot)
{
    constexpr int T = 1024, CH = kScanChunk8k;
    __shared__ uint32_t ws[T / 64];
    const int64_t nc0 = (nbins0 + CH - 1) / CH;
    const int arr = (int64_t)blockIdx.x < nc0 ? 0 : 1;
    const int64_t base = (arr ? (int64_t)blockIdx.x - nc0 : (int64_t)blockIdx.x) * CH;
    const uint32_t* __restrict__ totals = arr ? totals1 : totals0;
    const int64_t nbins = arr ? nbins1 : nbins0;
    uint32_t v = 0;
    for (int64_t i = base + threadIdx.x; i < base + CH && i < nbins; i += T) v += totals[i];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
    if ((threadIdx.x & 63) == 0) ws[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t t = 0;
        for (int i = 0; i < T / 64; ++i) t += ws[i];
        chunk_tot[blockIdx.x] = t;
    }
}

__global__ __launch_bounds__(1024) void scan_chunks_kernel(
    const uint32_t* __restrict__ totals0, int64_t nbins0, uint32_t* __restrict__ start0,
    uint32_t* __restrict__ occ0, uint32_t* __restrict__ occ0_n,
    const uint32_t* __restrict__ totals1, int64_t nbins1, uint32_t* __restrict__ start1,
    uint32_t* __restrict__ occ1, uint32_t* __restrict__ occ1_n,
    const uint32_t* __restrict__ chunk_tot)
{
    constexpr int T = 1024, K = 8, CH = kScanChunk8k, NWV = T / 64;
    static_assert(T * K == CH, "one chunk per workgroup");
    __shared__ uint32_t buf[CH];
    __shared__ uint32_t wsum[4][NWV];
    __shared__ uint32_t res[4];
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const int64_t nc0 = (nbins0 + CH - 1) / CH;
    const int arr = (int64_t)blockIdx.x < nc0 ? 0 : 1;
    const int64_t chunk = arr ? (int64_t)blockIdx.x - nc0 : (int64_t)blockIdx.x;
    const uint32_t* __restrict__ totals = arr ? totals1 : totals0;
    const int64_t nbins = arr ? nbins1 : nbins0;
    uint32_t* __restrict__ start = arr ? start1 : start0;
    uint32_t* __restrict__ list = arr ? occ1 : occ0;
    uint32_t* __restrict__ ln = arr ? occ1_n : occ0_n;
    const uint32_t cap = (uint32_t)nbins;
    const bool empties = arr != 0;
    const int64_t base = chunk * CH;
    // the chunk's own totals, and the sum of those before it
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const int64_t i = base + k * T + tid;
        buf[k * T + tid] = i < nbins ? totals[i] : 0u;
    }
    uint32_t before = 0;
    if (chunk_tot) {
        const int64_t c0 = arr ? nc0 : 0;
        for (int64_t c = tid; c < chunk; c += T) before += chunk_tot[c0 + c];
    } else {
        for (int64_t i = tid; i < base; i += T) before += totals[i];
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) before += __shfl_down(before, o, 64);
    if (lane == 0) wsum[0][wid] = before;
    if (tid == 0 && chunk == 0) ln[3] = cap;
    __syncthreads();
    uint32_t carry = 0;
#pragma unroll
    for (int i = 0; i < NWV; ++i) carry += wsum[0][i];
    const int64_t i0 = base + (int64_t)tid * K;
    // per thread: the sum, its listed light bins, and its heavy bins packed
    // (very heavy in the low 16 bits, heavy in the high 16: at most 512 of
    // either in a wavefront)
    uint32_t v[K], sum = 0, fsum = 0, h = 0;
#pragma unroll
    for (int k = 0; k < K; ++k) {
        v[k] = buf[tid * K + k];
        sum += v[k];
        if (v[k] >= kVeryHeavyBin) h += 1u;
        else if (v[k] >= kHeavyBin) h += 1u << 16;
        else if (i0 + k < nbins && (v[k] || empties)) ++fsum;
    }
    uint32_t x = sum, fx = fsum, hx = h;               // inclusive scans within the wave
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t y = __shfl_up(x, o, 64);
        const uint32_t fy = __shfl_up(fx, o, 64);
        const uint32_t hy = __shfl_up(hx, o, 64);
        if (lane >= o) {
            x += y;
            fx += fy;
            hx += hy;
        }
    }
    __syncthreads();        // (wsum[0] read above)
    if (lane == 63) {
        wsum[0][wid] = x;
        wsum[1][wid] = fx;
        wsum[2][wid] = hx & 0xffffu;
        wsum[3][wid] = hx >> 16;
    }
    __syncthreads();
    if (tid < 4) {
        // exclusive prefix over the wavefronts, and the chunk's entries of
        // each listed class reserved in the list
        uint32_t t = 0;
#pragma unroll
        for (int i = 0; i < NWV; ++i) {
            const uint32_t c = wsum[tid][i];
            wsum[tid][i] = t;
            t += c;
        }
        uint32_t r = 0;
        if (tid == 1 && t) r = atomicAdd(&ln[4], t);
        if (tid == 2 && t) r = atomicAdd(&ln[1], t);
        if (tid == 3 && t) r = atomicAdd(&ln[2], t);
        res[tid] = r;
        if (tid >= 1 && t) atomicAdd(&ln[0], t);
        if (tid == 0 && base + CH >= nbins) start[nbins] = carry + t;     // the array's end
    }
    __syncthreads();
    uint32_t run = carry + wsum[0][wid] + (x - sum);
    uint32_t frun = res[1] + wsum[1][wid] + (fx - fsum);
    uint32_t o2 = res[2] + wsum[2][wid] + ((hx - h) & 0xffffu);
    uint32_t o1 = res[3] + wsum[3][wid] + ((hx - h) >> 16);
#pragma unroll
    for (int k = 0; k < K; ++k) {
        buf[tid * K + k] = run;
        run += v[k];
        if (i0 + k < nbins) {
            const uint32_t bin = (uint32_t)(i0 + k);
            if (v[k] >= kVeryHeavyBin) list[2 * cap + o2++] = bin;
            else if (v[k] >= kHeavyBin) list[cap + o1++] = bin;
            else if (v[k] || empties) list[frun++] = bin;
        }
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const int64_t i = base + k * T + tid;
        if (i < nbins) start[i] = buf[k * T + tid];
    }
}

// In place: hist[b][bin] <- start[global bin] + sum_{b' < b} hist[b'][bin].
__global__ __launch_bounds__(256) void offsets_kernel(const WinMeta* __restrict__ meta, int nw,
                                                      int64_t ncells, int bwd,
                                                      uint32_t* __restrict__ hist,
                                                      const uint32_t* __restrict__ csum,
                                                      const uint32_t* __restrict__ start)
{
    const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= ncells) return;
    const int w = find_window(meta, nw, id,
                              [bwd](const WinMeta& m) { return BinSpace::cell_off(m, bwd); });
    const WinMeta& M = meta[w];
    const int nbins = BinSpace::nbins(M, bwd);
    const int64_t local = id - BinSpace::cell_off(M, bwd);
    const int c = (int)(local / nbins), bin = (int)(local - (int64_t)c * nbins);
    const int b0 = c * kScanChunk, nb = min(kScanChunk, M.G.nblocks - b0);
    uint32_t* h = hist + M.hist_off + (size_t)b0 * nbins + bin;
    // all of the chunk's counts are loaded before the first store (no serial
    // load-store chain down the column)
    uint32_t v[kScanChunk];
#pragma unroll
    for (int i = 0; i < kScanChunk; ++i) v[i] = i < nb ? h[(size_t)i * nbins] : 0u;
    uint32_t run = start[BinSpace::bin_off(M, bwd) + bin] + csum[M.csum_off + (size_t)c * nbins + bin];
#pragma unroll
    for (int i = 0; i < kScanChunk; ++i) {
        if (i < nb) h[(size_t)i * nbins] = run;
        run += v[i];
    }
}

// Writes each valid event's records into the slots its block reserved.
// Atomic mode: a record goes to every tile its taps reach, and each valid
// event's source record to its source bin(s) (see fwd_count); the block's
// LDS counters start at the bins' starts plus the block's offsets.
// Deterministic mode: the offsets kernel made the row absolute; the source
// record goes where the event's reference-0 record goes, relative to the
// window's first reference-0 slot.
template <int RM, int NT, bool DET, int FM>
__global__ __launch_bounds__(NT) void fwd_scatter_kernel(
    const WinMeta* __restrict__ meta, int nw, const int* __restrict__ win_of, const float* __restrict__ ex,
    const float* __restrict__ ey, const float* __restrict__ et, const int8_t* __restrict__ ep,
    const float* __restrict__ rho, const float* __restrict__ ego, const Motion* __restrict__ mtab,
    const uint32_t* __restrict__ offs, const uint32_t* __restrict__ start,
    const uint32_t* __restrict__ start_src, int ae, const uint8_t* __restrict__ valid,
    SplatRec* __restrict__ rec, SrcRec* __restrict__ src)
{
    extern __shared__ uint32_t lh[];
    const int64_t blk = xcd_block();
    const int w = win_of[blk];
    const WinParams& P = meta[w].P;
    const TileGeom G = meta[w].G;
    const int64_t lb = blk - meta[w].blk_off;
    const int64_t ev0 = meta[w].ev_off, n = meta[w].n;
    const int nrb = G.nbins;
    const int nlb = DET ? nrb : nrb + G.nbins_s;
    const uint32_t* row = offs + meta[w].hist_off + lb * nlb;
    __shared__ RefTable rt;
    for (int i = threadIdx.x; i < nlb; i += blockDim.x) {
        if (DET) lh[i] = row[i];
        else lh[i] = row[i] + (i < nrb ? start[meta[w].bin_off + i]
                                        : start_src[meta[w].sbin_off + (i - nrb)]);
    }
    load_ref_table(P, nullptr, rt);
    __shared__ MotionTable mt;
    const Flows<FM> u = make_flows_tab<FM>(P, rho + meta[w].pix_off, ego + 6 * meta[w].ego_off,
                                           mtab + meta[w].ego_off, &mt);
    __syncthreads();
    // deterministic mode: the window's reference-0 records come first among
    // its records, so their slots minus this offset number its valid events
    const uint32_t r0 = DET ? start[meta[w].bin_off] : 0u;
    SrcRec* wsrc = DET ? src + ev0 : src;
    const int64_t base = lb * NT * G.ept;
    const uint8_t* wvalid = valid + ev0;
    EventPrefetch nx(ex + ev0, ey + ev0, et + ev0, ep + ev0, base + threadIdx.x, n);
    uint8_t vn = base + threadIdx.x < n ? wvalid[base + threadIdx.x] : (uint8_t)0;
    for (int e = 0; e < G.ept; ++e) {
        const int64_t k = base + (int64_t)e * NT + threadIdx.x;
        if (k >= n) break;
        const EventPrefetch::Ev cur = nx.take(e + 1 < G.ept ? k + NT : n);
        const uint8_t vk = vn;
        if (e + 1 < G.ept && k + NT < n) vn = wvalid[k + NT];
        // The count kernel's warp of this event masked it or not; the same
        // warp here (same code, same inputs, no contraction: the same bits)
        // reaches the same visits, so a valid event's records are written as
        // its visits are reached, into the slots its counts reserved.
        if (!vk) continue;
        const float xk = cur.x, yk = cur.y, tk = cur.t;
        const float ts = cur.p > 0 ? fabsf(tk) : -fabsf(tk);   // sign bit = polarity
        SrcRec o;
        o.x0 = xk;
        o.y0 = yk;
        o.ts = ts;
        o.k = (uint32_t)k;
        if (!DET && ae)
            for_each_reached(tiles_reached(G, make_taps(P, xk, yk)), G.ntx, [&](int t) {
                store_nt(src + atomicAdd(&lh[nrb + t], 1u), o);
            });
        Visits v;
        warp_visits_v<RM, FM>(P, u, rt, xk, yk, tk, v, [&](int, double X, double Y, int r) {
            const Taps tp = make_taps(P, X, Y);
            SplatRec q;
            q.X = X;
            q.Y = Y;
            q.ts = ts;
            q.k = (uint32_t)k;
            if (DET) {
                const uint32_t slot = stable_slot(lh, r * G.ntiles + tile_index(G, tp));
                rec[slot] = q;
                if (r == 0) wsrc[slot - r0] = o;
            } else {
                const uint32_t tr = tiles_reached(G, tp);
                for_each_reached(tr + (uint32_t)(r * G.ntiles), G.ntx,
                                 [&](int b) { rec[atomicAdd(&lh[b], 1u)] = q; });
                if (r == 0 && !ae) store_nt(src + atomicAdd(&lh[nrb + (int)(tr & 0xffffu)], 1u), o);
            }
        });
    }
}

// ---------------------------------------------------------------------------
// Forward tile kernels
// ---------------------------------------------------------------------------

__device__ __forceinline__ void reduce_pixel(double2 a, double2 b, double eps, double& sum,
                                             double& cnt)
{
    if (a.x + b.x > 0.0) cnt += 1.0;
    if (a.x != 0.0 || a.y != 0.0) {
        const double T = a.y / (a.x + eps);
        sum += T * T;
    }
    if (b.x != 0.0 || b.y != 0.0) {
        const double T = b.y / (b.x + eps);
        sum += T * T;
    }
}

__device__ __forceinline__ void split_bin(const TileGeom& G, int bin, int& r, int& tx, int& ty)
{
    r = bin / G.ntiles;
    const int tile = bin - r * G.ntiles;
    ty = tile / G.ntx;
    tx = tile - ty * G.ntx;
}

__device__ __forceinline__ int window_of_bin(const WinMeta* meta, int nw, int64_t gbin)
{
    return find_window(meta, nw, gbin, [](const WinMeta& m) { return m.bin_off; });
}

__device__ __forceinline__ int window_of_bbin(const WinMeta* meta, int nw, int64_t gbb)
{
    return find_window(meta, nw, gbb, [](const WinMeta& m) { return m.bbin_off; });
}

// Per-call preparation, one launch: the window of every event block, forward
// bin and backward bin of the batch (one binary search per entry per call
// instead of a chain of dependent loads at the start of every workgroup), the
// forward bins' records; (one thread per window) the first-order motion
// coefficients of every flow set and cleared per-window headers (hdrs,
// forward only); zeroed chunk sums.
// tab = [blocks | forward bins | backward bins].  Each block first copies the
// windows' first block, bin and backward bin into LDS (batches of up to
// kTableLdsWindows windows; larger ones search the metadata in memory), so
// that a search costs one global load instead of one per step.
constexpr int kTableLdsWindows = 512;
__global__ __launch_bounds__(256) void window_table_kernel(const WinMeta* __restrict__ meta,
                                                           int nw, int64_t nblk, int64_t nbin,
                                                           int64_t nbb, int* __restrict__ tab,
                                                           const float* __restrict__ ego,
                                                           Motion* __restrict__ mtab,
                                                           StateHeader* __restrict__ hdrs,
                                                           uint32_t* __restrict__ csum,
                                                           int64_t ncsum, TileBin* __restrict__ tbin,
                                                           double* __restrict__ zero2 = nullptr,
                                                           int64_t nzero2 = 0)
{
    __shared__ int64_t first[3][kTableLdsWindows];
    const bool lds = nw <= kTableLdsWindows;
    if (lds) {
        for (int w = threadIdx.x; w < nw; w += blockDim.x) {
            first[0][w] = meta[w].blk_off;
            first[1][w] = meta[w].bin_off;
            first[2][w] = meta[w].bbin_off;
        }
        __syncthreads();
    }
    // largest w with first[kind][w] <= key
    auto search = [&](int kind, int64_t key) {
        if (!lds) {
            if (kind == 0) return window_of_block(meta, nw, key);
            if (kind == 1) return window_of_bin(meta, nw, key);
            return window_of_bbin(meta, nw, key);
        }
        int lo = 0, hi = nw - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (first[kind][mid] <= key) lo = mid;
            else hi = mid - 1;
        }
        return lo;
    };
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < nblk) {
        tab[i] = search(0, i);
        return;
    }
    i -= nblk;
    if (i < nbin) {
        const int w = search(1, i);
        tab[nblk + i] = w;
        const WinParams& P = meta[w].P;
        int r, tx, ty;
        split_bin(meta[w].G, (int)(i - meta[w].bin_off), r, tx, ty);
        TileBin b;
        b.ref = P.refs[r];
        b.eps = P.eps;
        b.plane = meta[w].img_off + (int64_t)r * 2 * P.HW;
        b.W = P.W;
        b.H = P.H;
        b.xo = tx * meta[w].G.tw;
        b.yo = ty * meta[w].G.th;
        b.ntx = meta[w].G.ntx;
        b.pad = 0;
        tbin[i] = b;
        return;
    }
    i -= nbin;
    if (i < nbb) {
        tab[nblk + nbin + i] = search(2, i);
        return;
    }
    i -= nbb;
    if (i < nw) {
        const int w = (int)i;
        const WinParams& P = meta[w].P;
        for (int f = 0; f < P.F; ++f)
            mtab[meta[w].ego_off + f] = load_motion(P, ego + 6 * (meta[w].ego_off + f));
        if (hdrs) {
            StateHeader z;
            z.loss = 0.0;
            z.n_valid = 0;
            z.flags = 0;
            for (int r = 0; r < kMaxRefs; ++r) {
                z.num[r] = 0.0;
                z.nact[r] = 0.0;
            }
            hdrs[w] = z;
        }
        return;
    }
    i -= nw;
    if (i < ncsum) {
        csum[i] = 0u;
        return;
    }
    i -= ncsum;
    if (i < nzero2) zero2[i] = 0.0;
}

// Threads of the forward tile kernel: the deterministic mode keeps 256 (its
// reduction order is defined on them); the atomic mode uses more by default
// (a tuning), so that the blocks whose LDS tiles fit a CU keep more
// wavefronts in flight.
constexpr int kTileThreadsDet = 256;
constexpr int kTileThreads = 512;

// Deterministic mode: one workgroup per (reference, tile) bin accumulates its
// records in a 33 x 33 LDS tile (the tile and its right column / bottom row
// halo) in record order; column 0 and row 0 go to a border buffer and the
// halo to a halo buffer, which the merge combines in a fixed order.
//
// The order is per pixel: the bin's records 64 at a time, then tap slot 0..3,
// then lane.  kDetAccWaves wavefronts walk the records in that order
// together, each adding only the contributions to the LDS cells it owns
// (cell index mod kDetAccWaves): every cell is updated by one wavefront in
// the canonical order, so the bits are those of a single wavefront walking
// all of them, and the serial part (one pass per distinct cell of a slot)
// splits over the wavefronts.  The output and its reduction run on the first
// kTileThreadsDet threads, in the order the reduction is defined on.
constexpr int kDetAccWaves = 16;

__global__ __launch_bounds__(64 * kDetAccWaves) void fwd_tile_det_kernel(const TileBin* __restrict__ tbin,
                                                       const SplatRec* __restrict__ rec,
                                                       const uint32_t* __restrict__ start,
                                                       double2* __restrict__ img_base,
                                                       double2* __restrict__ halo,
                                                       double2* __restrict__ border,
                                                       double* __restrict__ part)
{
    __shared__ double2 lds[2 * TLW * TLH];
    // cells reached only by zero-weight taps (positions on a pixel row or
    // column): they hold zeros, but the backward reads them (see below)
    __shared__ uint32_t zbit[(2 * TLW * TLH + 31) / 32];
    __shared__ double red[32];
    const int64_t gbin = blockIdx.x;
    // the bin's bounds and its record, loaded together
    const uint32_t s0 = start[gbin], s1 = start[gbin + 1];
    const TileBin bi = tbin[gbin];
    if (s0 == s1) {
        // No warped position falls in this tile at this reference.  Nothing
        // reads its pixels except column 0 and row 0, which the merge writes
        // from the neighbours' halos; a backward gather at a tap of this tile
        // comes from a position binned in a left or upper neighbour, whose
        // taps reach only that column and row.  Its halo is not written
        // either: the merge reads halos of occupied bins only.  So only zero
        // sums are written (56% of the c3 bins are empty).
        if (threadIdx.x == 0) {
            part[(gbin * 2 + 0) * 2 + 0] = 0.0;
            part[(gbin * 2 + 0) * 2 + 1] = 0.0;
        }
        return;
    }
    const int xo = bi.xo, yo = bi.yo;
    for (int i = threadIdx.x; i < 2 * TLW * TLH; i += blockDim.x) lds[i] = make_double2(0.0, 0.0);
    for (int i = threadIdx.x; i < (2 * TLW * TLH + 31) / 32; i += blockDim.x) zbit[i] = 0u;
    __syncthreads();
    const double ref = bi.ref;
    {
        // every wavefront walks the records in order, 64 at a time; per tap
        // slot, equal cells among its own are updated in lane order
        const int wave = (int)(threadIdx.x >> 6);
        for (uint32_t b0 = s0; b0 < s1; b0 += 64) {
            const uint32_t i = b0 + __lane_id();
            const bool live = i < s1;
            SplatRec q;
            if (live) q = rec[i];
            else q.X = q.Y = (double)xo, q.ts = 0.f;
            const int pol = (__float_as_uint(q.ts) >> 31) ? 1 : 0;
            const double tb = 1.0 - fabs(ref - (double)fabsf(q.ts));
            const Taps tp = make_taps_wh(bi.W, bi.H, q.X, q.Y);
            const int lx = tp.x0 - xo, ly = tp.y0 - yo;
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                const double wt = tap_w(tp, c);
                const int key = pol * TLW * TLH + (ly + (c >> 1)) * TLW + lx + (c & 1);
                const bool mine = live && tap_in(tp, c) && key % kDetAccWaves == wave;
                if (mine && wt == 0.0) atomicOr(&zbit[key >> 5], 1u << (key & 31));
                ordered_add(lds, mine && wt != 0.0, key, wt, wt * tb);
            }
        }
    }
    __syncthreads();
    double sum = 0.0, cnt = 0.0;
    double2* plane0 = img_base + bi.plane;
    double2* plane1 = plane0 + (size_t)bi.W * bi.H;
    // Interior pixels to the image; column 0 and row 0 to the border buffer,
    // which the merge completes with the neighbours' halos and stores.  The
    // backward reads the image only at the taps of the positions splatted
    // here, and an interior pixel's taps all come from this bin's records: so
    // of the interior only the cells some tap reached are stored (a non-zero
    // sum, or a zero-weight tap's bit), the others are neither written nor
    // read.
    double2* fb = border + gbin * NBORDER * 2;
    auto reached = [&](int k, const double2& c) {
        return c.x != 0.0 || c.y != 0.0 || ((zbit[k >> 5] >> (k & 31)) & 1u);
    };
    for (int i = threadIdx.x; i < TW * TH && threadIdx.x < kTileThreadsDet; i += kTileThreadsDet) {
        const int lx = i % TW, ly = i / TW;
        const int X = xo + lx, Y = yo + ly;
        if (X >= bi.W || Y >= bi.H) continue;
        const int k = ly * TLW + lx;
        const double2 a = lds[k], b = lds[TLW * TLH + k];
        if (lx == 0 || ly == 0) {
            const int j = lx == 0 ? ly : TH + lx - 1;
            fb[j * 2 + 0] = a;
            fb[j * 2 + 1] = b;
            continue;
        }
        const int pix = Y * bi.W + X;
        if (reached(k, a)) plane0[pix] = a;
        if (reached(TLW * TLH + k, b)) plane1[pix] = b;
        reduce_pixel(a, b, bi.eps, sum, cnt);
    }
    double2* hb = halo + gbin * NHALO * 2;
    for (int j = threadIdx.x; j < NHALO; j += blockDim.x) {
        const int idx = (j <= TH) ? j * TLW + TW : TH * TLW + (j - (TH + 1));
        hb[j * 2 + 0] = lds[idx];
        hb[j * 2 + 1] = lds[TLW * TLH + idx];
    }
    double sc[2] = {sum, cnt};
    block_sum_n(sc, red, kTileThreadsDet / 64);
    if (threadIdx.x == 0) {
        part[(gbin * 2 + 0) * 2 + 0] = sc[0];
        part[(gbin * 2 + 0) * 2 + 1] = sc[1];
    }
}

// One wavefront's sum (lanes in the shuffle-down tree of block_sum; the
// result, valid in lane 0, is 0.0 + the tree's value as block_sum gives it
// for a one-wavefront block).
__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
    return 0.0 + v;
}

// A double moved across lanes by a DPP control (both halves; lanes with no
// source lane get 0).
template <int CTRL, int ROWS>
__device__ __forceinline__ double dpp_f64(double v)
{
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, ROWS, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, ROWS, 0xf, false);
    return __hiloint2double(hi, lo);
}

// One wavefront's sum by DPP moves (no LDS round trips), valid in lane 63:
// prefix sums within each row of 16 lanes (row_shr 1, 2, 4, 8), then row
// 15's value broadcast into the next row (row_bcast:15) and lane 31's into
// the upper half (row_bcast:31).  Where the additions fall differs from
// wave_sum (any order: the atomic mode's sums are not order-fixed).
__device__ __forceinline__ double wave_sum_dpp(double v)
{
    v += dpp_f64<0x111, 0xf>(v);     // row_shr:1
    v += dpp_f64<0x112, 0xf>(v);     // row_shr:2
    v += dpp_f64<0x114, 0xf>(v);     // row_shr:4
    v += dpp_f64<0x118, 0xf>(v);     // row_shr:8
    v += dpp_f64<0x142, 0xa>(v);     // row_bcast:15 into rows 1 and 3
    v += dpp_f64<0x143, 0xc>(v);     // row_bcast:31 into rows 2 and 3
    return v;
}

// Partial sums of Eq. 1 per forward bin in the atomic mode: one (sum, count)
// pair per wavefront of the splat workgroup (at most 8), so that a bin needs
// no cross-wavefront reduction; the finalize adds them.
constexpr int kPartOwn = 16;

// A splat workgroup's table of its bins (list entry, bounds, table entry),
// loaded kBinTable at a time.
constexpr int kBinTable = 64;
struct OwnBin {
    TileBin b;
    uint32_t g, s0, s1, pad;
};

// Atomic mode: a (reference, tile) bin owns the tile's pixels (TWX x THX, the
// plan's tile size; 32 x 32 by default).  Its bin holds every record whose
// taps reach the tile (its own positions and the copies from the left, upper
// and upper-left neighbours), so its workgroup accumulates the taps that fall
// in the tile with FP64 LDS atomics, stores the pixels some tap reached and
// reduces Eq. 1 over all its pixels: no halo, no merge.  Only occupied bins
// are visited (the scan lists them; the window table kernel zeroed the
// partial sums of the others).  The list runs heaviest first and the grid is
// what fits the chip at once, ncu CUs x per_cu workgroups, workgroup b on CU
// b mod ncu (the dispatcher's order).  The list is dealt out in passes of one
// bin per CU, alternating direction (pass p gives entry p ncu + c, or
// p ncu + ncu - 1 - c on odd passes, to CU c), and the CU's workgroup b / ncu
// takes passes b / ncu, b / ncu + per_cu, ...: the longest bins start at
// once, on different CUs, and the CUs' sums even out.  Per bin the chain is:
// accumulate, barrier, output, barrier.
// - The workgroup's list entries, bin bounds and table entries are loaded
//   into LDS up front (kBinTable bins at a time), so that no scalar load is
//   in flight in the loop: scalar loads share the LDS operations' counter,
//   and the next LDS wait would wait for them.
// - The next bin's records are loaded right after the accumulation barrier,
//   in flight during the output.
// - The output loop reads, stores and clears only the cells some tap reached
//   (a byte per cell marks them), so the next bin starts on a clear tile
//   with no clearing pass (the tile is cleared once, up front).
// - Each wavefront reduces its pixels' Eq. 1 terms and writes its own pair
//   of partial sums: no block reduction and its two barriers.
// C and S accumulate in separate LDS arrays (8-byte stride: half the bank
// conflicts of interleaved pairs).
template <int NTT, int TWX, int THX>
__global__ __launch_bounds__(NTT) void fwd_tile_own_kernel(const TileBin* __restrict__ tbin,
                                                           const SplatRec* __restrict__ rec,
                                                           const uint32_t* __restrict__ start,
                                                           const uint32_t* __restrict__ occ,
                                                           const uint32_t* __restrict__ occ_n,
                                                           double2* __restrict__ img_base,
                                                           double* __restrict__ part, int ncu)
{
    static_assert(NTT / 64 * 2 <= kPartOwn, "one partial pair per wavefront");
    static_assert(NTT >= kBinTable, "one table entry per thread");
    constexpr int NPIX = TWX * THX;
    __shared__ double lc[2 * NPIX];       // C by polarity, then pixel
    __shared__ double ls[2 * NPIX];       // S
    // cells some tap reached (positive or zero weight: a position on a pixel
    // row or column gives zero-weight taps, whose pixels hold zeros but are
    // read by the backward)
    __shared__ uint8_t tch[2 * NPIX];
    __shared__ OwnBin tab[kBinTable];
    const uint32_t nocc = occ_n[0];
    const uint32_t G = gridDim.x;
    if (nocc == 0) return;
    const uint32_t nc = (uint32_t)ncu, per = G / nc;
    const uint32_t slot = blockIdx.x / nc, cu = blockIdx.x - slot * nc;
    // list entry of pass p for this CU
    auto entry = [&](uint32_t p) { return p * nc + ((p & 1) ? nc - 1 - cu : cu); };
    // this workgroup's bins: its passes among the full ones, and the partial
    // last pass if it is one of its passes and reaches its CU
    const uint32_t pf = nocc / nc;
    uint32_t nb = pf > slot ? (pf - slot - 1) / per + 1 : 0u;
    if (pf % per == slot && entry(pf) < nocc) ++nb;
    if (nb == 0) return;
    auto load_table = [&](uint32_t j0) {
        const uint32_t j = j0 + threadIdx.x;
        if (threadIdx.x < kBinTable && j < nb) {
            OwnBin e;
            const uint32_t kk = entry(j * per + slot);
            e.g = kk < nocc ? occ_entry(occ, occ_n, kk) : 0u;
            e.s0 = start[e.g];
            e.s1 = start[e.g + 1];
            e.b = tbin[e.g];
            e.pad = 0;
            tab[threadIdx.x] = e;
        }
    };
    load_table(0);
    for (int i = threadIdx.x; i < 2 * NPIX; i += NTT) {
        lc[i] = 0.0;
        ls[i] = 0.0;
        tch[i] = 0;
    }
    __syncthreads();
    SplatRec qq[2];
    auto load_first = [&](uint32_t a0, uint32_t a1) {
        const uint32_t i0 = a0 + threadIdx.x;
        if (i0 < a1) {
            qq[0] = rec[i0];
            qq[1] = rec[i0 + NTT < a1 ? i0 + NTT : i0];
        }
    };
    load_first(tab[0].s0, tab[0].s1);
    for (uint32_t j = 0;;) {
        const OwnBin& e = tab[j % kBinTable];
        const uint32_t gbin = e.g, s0 = e.s0, s1 = e.s1;
        const TileBin bi = e.b;
        const int xo = bi.xo, yo = bi.yo;
        const double ref = bi.ref;
        for (uint32_t i0 = s0 + threadIdx.x; i0 < s1;) {
            const bool two = i0 + NTT < s1;
#pragma unroll
            for (int u = 0; u < 2; ++u) {
                if (u == 1 && !two) break;
                const SplatRec q = qq[u];
                const int pol = (__float_as_uint(q.ts) >> 31) ? 1 : 0;
                const double tb = 1.0 - fabs(ref - (double)fabsf(q.ts));
                const Taps tp = make_taps_wh(bi.W, bi.H, q.X, q.Y);
                const int lx = tp.x0 - xo, ly = tp.y0 - yo;
#pragma unroll
                for (int c = 0; c < 4; ++c) {
                    const int cx = lx + (c & 1), cy = ly + (c >> 1);
                    if (!tap_in(tp, c) || (unsigned)cx >= (unsigned)TWX ||
                        (unsigned)cy >= (unsigned)THX)
                        continue;
                    const double wt = tap_w(tp, c);
                    const int key = pol * NPIX + cy * TWX + cx;
                    tch[key] = 1;
                    if (wt == 0.0) continue;
                    atomicAdd(&lc[key], wt);
                    atomicAdd(&ls[key], wt * tb);
                }
            }
            i0 += 2 * NTT;
            if (i0 < s1) {
                qq[0] = rec[i0];
                qq[1] = rec[i0 + NTT < s1 ? i0 + NTT : i0];
            }
        }
        __syncthreads();
        const uint32_t jn = j + 1;
        // the next bin's first records, in flight during the output (at a
        // table boundary they wait for the next table)
        if (jn < nb && jn % kBinTable != 0) load_first(tab[jn % kBinTable].s0, tab[jn % kBinTable].s1);
        double sum = 0.0, cnt = 0.0;
        double2* plane0 = img_base + bi.plane;
        double2* plane1 = plane0 + (size_t)bi.W * bi.H;
        // The backward reads the image only at the taps of the positions
        // splatted here, and every such tap reached this tile through its
        // bin: so only the pixels some tap reached are stored, the others are
        // neither written nor read.  Untouched cells hold zeros and add
        // nothing to Eq. 1: they are skipped.
        for (int i = threadIdx.x; i < NPIX; i += NTT) {
            const bool ta = tch[i] != 0, tb2 = tch[NPIX + i] != 0;
            if (!ta && !tb2) continue;
            double2 a = make_double2(0.0, 0.0), b = make_double2(0.0, 0.0);
            if (ta) {
                a = make_double2(lc[i], ls[i]);
                lc[i] = 0.0;
                ls[i] = 0.0;
                tch[i] = 0;
            }
            if (tb2) {
                b = make_double2(lc[NPIX + i], ls[NPIX + i]);
                lc[NPIX + i] = 0.0;
                ls[NPIX + i] = 0.0;
                tch[NPIX + i] = 0;
            }
            // (taps off the sensor are never made: a touched cell is on it)
            const int pix = (yo + i / TWX) * bi.W + xo + (i % TWX);
            if (ta) plane0[pix] = a;
            if (tb2) plane1[pix] = b;
            reduce_pixel(a, b, bi.eps, sum, cnt);
        }
        sum = wave_sum_dpp(sum);
        cnt = wave_sum_dpp(cnt);
        if ((threadIdx.x & 63) == 63) {
            double* pp = part + (size_t)gbin * kPartOwn + (threadIdx.x >> 6) * 2;
            pp[0] = sum;
            pp[1] = cnt;
        }
        if (jn >= nb) break;
        __syncthreads();        // the cleared tile (and the read table), for the next bin
        j = jn;
        if (j % kBinTable == 0) {
            load_table(j);
            __syncthreads();
            load_first(tab[0].s0, tab[0].s1);
        }
    }
}

// Column 0 and row 0 of each tile: the tile's own values (border buffer) plus
// the halos of the left, top and top-left tiles (in that order); store and
// reduce those pixels.

// One wavefront per bin, kMergeBins bins per block (the bins are
// independent: no barrier).
constexpr int kMergeBins = 4;

__global__ __launch_bounds__(64 * kMergeBins) void fwd_merge_kernel(const TileBin* __restrict__ tbin, int64_t nbins,
                                                       const uint32_t* __restrict__ start,
                                                       double2* __restrict__ img_base,
                                                       const double2* __restrict__ halo,
                                                       const double2* __restrict__ border,
                                                       double* __restrict__ part)
{
    const int64_t gbin = (int64_t)blockIdx.x * kMergeBins + (threadIdx.x >> 6);
    if (gbin >= nbins) return;
    const int lane = threadIdx.x & 63;
    const TileBin bi = tbin[gbin];     // the bin's geometry without a window lookup
    const int xo = bi.xo, yo = bi.yo, tx = xo / TW, ty = yo / TH;
    const int64_t HW = (int64_t)bi.W * bi.H;
    // occupied bins (the tile kernel wrote their border and halo); an empty
    // bin whose left, upper and upper-left neighbours are empty too has a
    // zero border that no gather reads: nothing to write
    auto occupied = [&](int64_t b) { return start[b] != start[b + 1]; };
    const bool own = occupied(gbin);
    const bool left = tx > 0 && occupied(gbin - 1);
    const bool up = ty > 0 && occupied(gbin - bi.ntx);
    const bool upleft = tx > 0 && ty > 0 && occupied(gbin - bi.ntx - 1);
    if (!(own || left || up || upleft)) {
        if (lane == 0) {
            part[(gbin * 2 + 1) * 2 + 0] = 0.0;
            part[(gbin * 2 + 1) * 2 + 1] = 0.0;
        }
        return;
    }
    double sum = 0.0, cnt = 0.0;
    for (int j = lane; j < NBORDER; j += 64) {
        const int lx = j < TH ? 0 : j - TH + 1;
        const int ly = j < TH ? j : 0;
        const int X = xo + lx, Y = yo + ly;
        if (X >= bi.W || Y >= bi.H) continue;
        const int pix = Y * bi.W + X;
        double2 v[2];
#pragma unroll
        for (int pol = 0; pol < 2; ++pol) {
            double2 a = own ? border[(gbin * NBORDER + j) * 2 + pol] : make_double2(0.0, 0.0);
            if (lx == 0 && left) {
                const double2 h = halo[((gbin - 1) * NHALO + ly) * 2 + pol];
                a.x += h.x;
                a.y += h.y;
            }
            if (ly == 0 && up) {
                const double2 h = halo[((gbin - bi.ntx) * NHALO + TH + 1 + lx) * 2 + pol];
                a.x += h.x;
                a.y += h.y;
            }
            if (lx == 0 && ly == 0 && upleft) {
                const double2 h = halo[((gbin - bi.ntx - 1) * NHALO + TH) * 2 + pol];
                a.x += h.x;
                a.y += h.y;
            }
            img_base[bi.plane + pol * HW + pix] = a;
            v[pol] = a;
        }
        reduce_pixel(v[0], v[1], bi.eps, sum, cnt);
    }
    sum = wave_sum(sum);
    cnt = wave_sum(cnt);
    if (lane == 0) {
        part[(gbin * 2 + 1) * 2 + 0] = sum;
        part[(gbin * 2 + 1) * 2 + 1] = cnt;
    }
}

// One block per window: fixed-order sums of the tile and merge partials per
// reference, then Eq. 1.
// One workgroup per window: Eq. 1 per reference from its bins' partial sums
// (pstride doubles per bin, of which the first pused (sum, count) pairs are
// written: one per wavefront of the atomic mode's splat workgroup, two in the
// deterministic mode), then the loss.  The atomic mode gives each reference
// a wavefront of its own (per_wave; 64 R threads); the deterministic mode
// takes the references in turn over 256 threads (its fixed addition order).
constexpr int kFinalizeThreads = 1024;
__global__ __launch_bounds__(kFinalizeThreads) void fwd_finalize_kernel(
    const WinMeta* __restrict__ meta, const double* __restrict__ part, int pstride, int pused,
    int per_wave, StateHeader* __restrict__ hdrs, float* __restrict__ loss)
{
    __shared__ double red[16 * 2];
    const int w = blockIdx.x;
    const WinParams& P = meta[w].P;
    const TileGeom G = meta[w].G;
    const double* pw = part + meta[w].bin_off * pstride;
    const int nt = G.ntiles * pused;
    StateHeader* hdr = hdrs + w;
    double L = 0.0;
    if (per_wave) {
        // atomic mode: wavefront r sums reference r's partials (R <= 16
        // wavefronts), one barrier for all
        const int lane = threadIdx.x & 63, r = threadIdx.x >> 6;
        double a = 0.0, b = 0.0;
        if (r < P.R) {
            const double* pr = pw + (size_t)r * G.ntiles * pstride;
            // eight items per lane and round, loaded before they are added
            for (int t0 = lane; t0 < nt; t0 += 8 * 64) {
                double2 v[8];
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    const int t = t0 + u * 64;
                    v[u] = make_double2(0.0, 0.0);
                    if (t < nt) {
                        const int tile = t / pused, q = t - tile * pused;
                        const double* pp = pr + (size_t)tile * pstride + 2 * q;
                        v[u] = make_double2(pp[0], pp[1]);
                    }
                }
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    a += v[u].x;
                    b += v[u].y;
                }
            }
        }
        a = wave_sum_dpp(a);
        b = wave_sum_dpp(b);
        if (lane == 63) {
            red[2 * r] = a;
            red[2 * r + 1] = b;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            for (int q = 0; q < P.R; ++q) {
                hdr->num[q] = red[2 * q];
                hdr->nact[q] = red[2 * q + 1];
                L += red[2 * q] / (red[2 * q + 1] + P.eps);
            }
            L = L / (double)P.R;
            hdr->loss = L;
            hdr->flags = kHdrSourceRecords;
            loss[w] = (float)L;
        }
        return;
    }
    for (int r = 0; r < P.R; ++r) {
        double sc[2] = {0.0, 0.0};
        // four items per round, loaded before they are added (in item order:
        // the same additions as one item at a time)
        const int nthr = (int)blockDim.x;
        for (int t0 = threadIdx.x; t0 < nt; t0 += 4 * nthr) {
            double2 v[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int t = t0 + u * nthr;
                v[u] = make_double2(0.0, 0.0);
                if (t < nt) {
                    const int tile = t / pused, q = t - tile * pused;
                    const double* pp = pw + ((size_t)r * G.ntiles + tile) * pstride + 2 * q;
                    v[u] = make_double2(pp[0], pp[1]);
                }
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                if (t0 + u * nthr < nt) {
                    sc[0] += v[u].x;
                    sc[1] += v[u].y;
                }
            }
        }
        block_sum_n(sc, red);
        if (threadIdx.x == 0) {
            hdr->num[r] = sc[0];
            hdr->nact[r] = sc[1];
            L += sc[0] / (sc[1] + P.eps);
        }
    }
    if (threadIdx.x == 0) {
        L = L / (double)P.R;
        hdr->loss = L;
        hdr->flags = kHdrSourceRecords;
        loss[w] = (float)L;
    }
}

// ---------------------------------------------------------------------------
// Backward: one record per flow-sampling position.  The forward sweep into
// reference r samples the flow at the previous position (the event for the
// first step), the backward sweep likewise; both first steps sample at the
// event, so their contributions share one record.
// ---------------------------------------------------------------------------

// The flow-sampling positions of an event's warp steps, with the flow set of
// each step: the previous visit's position for every real step that does not
// start at the event, and the event for the steps that do.  A window with one
// flow set has both sweeps' first steps share one event record; with several,
// each step has its own record (its set may differ).  Which of the two is
// decided per window, so a one-flow window gives the same records in any
// batch.
template <int RM, int FM, typename F>
__device__ __forceinline__ void for_each_sample(const WinParams& P, const RefTable& rt,
                                                const Visits& v, const uint32_t (&tl)[RM],
                                                uint32_t tev, F&& fn)
{
    // tl[j]: tile of visit j's position; tev: tile of the event.  A visit's
    // reference is mb + j in the forward sweep, mb - 1 - (j - nf) backward.
    const int jf = v.eq ? 1 : 0;
    if (FM != 0 && P.F > 1) {
#pragma unroll
        for (int j = 0; j < RM; ++j) {
            if (j < P.R && !(v.eq && j == 0)) {
                const bool first = (j == jf && j < v.nf) || (j == v.nf);
                const int set = j < v.nf ? rt.sf[v.mb + j] : rt.sb[v.mb - 1 - (j - v.nf)];
                fn(first ? tev : tl[j > 0 ? j - 1 : 0], set);
            }
        }
    } else {
#pragma unroll
        for (int j = 1; j < RM; ++j)
            if (j < P.R && j != jf && j != v.nf) fn(tl[j - 1], 0);
        if (P.R - jf > 0) fn(tev, 0);
    }
}

// The backward's event blocks run over the source records (valid events in
// reference-0 tile order) instead of the raw events, with the same block
// geometry, interleaved: in iteration e, block b of a window takes source
// positions [(e * nblocks + b) * NT, +NT).  The blocks in flight then work on
// one compact stretch of the source order, that is on neighbouring tiles, and
// their image and inverse-depth gathers share the L2.
//
// The window's source records: deterministic mode, [ev_off, ev_off + n_valid)
// of src; atomic mode, the window's source bins.  None (n = 0) if the forward
// was not the tiled one.
struct SrcRange {
    const SrcRec* p;
    int64_t n;
};

template <bool DET>
__device__ __forceinline__ SrcRange src_range(const WinMeta& M, const StateHeader& h,
                                              const SrcRec* src, const uint32_t* start_src)
{
    SrcRange s;
    if (!(h.flags & kHdrSourceRecords)) {
        s.p = src;
        s.n = 0;
    } else if (DET) {
        s.p = src + M.ev_off;
        s.n = (int64_t)h.n_valid;
    } else {
        const uint32_t a = start_src[M.sbin_off], b = start_src[M.sbin_off + M.G.nbins_s];
        s.p = src + a;
        s.n = (int64_t)(b - a);
    }
    return s;
}

template <int RM, int NT, int FM, bool DET>
__global__ __launch_bounds__(NT, 3) void bwd_count_kernel(
    const WinMeta* __restrict__ meta, int nw, const int* __restrict__ win_of, const SrcRec* __restrict__ src,
    const uint32_t* __restrict__ start_src, const float* __restrict__ rho,
    const float* __restrict__ ego, const Motion* __restrict__ mtab,
    const StateHeader* __restrict__ hdrs, uint32_t* __restrict__ hist, uint32_t* __restrict__ csum,
    uint32_t* __restrict__ totals)
{
    extern __shared__ uint32_t lh[];
    __shared__ uint32_t tls[RM][NT];
    const int64_t blk = xcd_block();
    const int w = win_of[blk];
    const WinParams& P = meta[w].P;
    const TileGeom G = meta[w].G;
    const int64_t lb = blk - meta[w].blk_off;
    const SrcRange sr = src_range<DET>(meta[w], hdrs[w], src, start_src);
    const int64_t nv = sr.n;
    const SrcRec* wsrc = sr.p;
    __shared__ RefTable rt;
    for (int i = threadIdx.x; i < G.nbins_b; i += blockDim.x) lh[i] = 0;
    load_ref_table(P, nullptr, rt);
    __shared__ MotionTable mt;
    const Flows<FM> u = make_flows_tab<FM>(P, rho + meta[w].pix_off, ego + 6 * meta[w].ego_off,
                                           mtab + meta[w].ego_off, &mt);
    __syncthreads();
    const int64_t stride = (int64_t)G.nblocks * NT;
    // One flow and references {0, 1} (or a single reference): every warp step
    // starts at the event, so the sweep's records all sit at the events' own
    // positions (one per valid event, none for an event on the single
    // reference) and the bins need no warp.  Source records exist for valid
    // events only.
    const bool at_events = !(FM != 0 && P.F > 1) &&
                           (P.R == 1 || (P.R == 2 && rt.t[0] == 0.0 && rt.t[1] == 1.0));
    // a sampling position's bin (deterministic) or bins (atomic: every tile
    // its taps reach)
    auto add = [&](uint32_t t, int set) {
        if (DET) atomicAdd(&lh[set * G.ntiles + (int)t], 1u);
        else for_each_reached(t + (uint32_t)(set * G.ntiles), G.ntx,
                              [&](int b) { atomicAdd(&lh[b], 1u); });
    };
    auto tile_of = [&](double X, double Y) -> uint32_t {
        const Taps tp = make_taps(P, X, Y);
        return DET ? (uint32_t)tile_index(G, tp) : tiles_reached(G, tp);
    };
    SrcRec qn;
    int64_t i = (int64_t)lb * NT + threadIdx.x;
    if (i < nv) qn = load_nt(wsrc + i);
    for (int e = 0; e < G.ept; ++e, i += stride) {
        if (i >= nv) break;
        const SrcRec q = qn;
        if (e + 1 < G.ept && i + stride < nv) qn = load_nt(wsrc + i + stride);
        const double x0 = q.x0, y0 = q.y0, tk = fabsf(q.ts);
        if (at_events) {
            if (!(P.R == 1 && rt.t[0] == tk)) add(tile_of(x0, y0), 0);
            continue;
        }
        // each visit's tile, in the thread's LDS column (see fwd_count)
        Visits v;
        if (!warp_visits_v<RM, FM>(P, u, rt, x0, y0, tk, v,
                                   [&](int j, double X, double Y, int) {
                                       tls[j][threadIdx.x] = tile_of(X, Y);
                                   }))
            continue;
        uint32_t tl[RM];
#pragma unroll
        for (int j = 0; j < RM; ++j) tl[j] = j < P.R ? tls[j][threadIdx.x] : 0u;
        for_each_sample<RM, FM>(P, rt, v, tl, tile_of(x0, y0),
                                [&](uint32_t tile, int set) { add(tile, set); });
    }
    __syncthreads();
    uint32_t* row = hist + meta[w].hist_off + lb * G.nbins_b;
    if (DET) {
        uint32_t* cs = csum + meta[w].csum_off + (size_t)(lb / kScanChunk) * G.nbins_b;
        for (int i = threadIdx.x; i < G.nbins_b; i += blockDim.x) {
            const uint32_t c = lh[i];
            row[i] = c;
            if (c) atomicAdd(cs + i, c);
        }
    } else {
        for (int i = threadIdx.x; i < G.nbins_b; i += blockDim.x) {
            const uint32_t c = lh[i];
            row[i] = c ? atomicAdd(totals + (meta[w].bbin_off + i), c) : 0u;
        }
    }
}

// Re-runs each valid event's warp, gathers the adjoint seeds, runs the
// reverse sweep and emits one record (sampling position, dt * adjoint) per
// flow-sampling position.  Deterministic mode: into the position's bin, at
// the slot stable_slot gives.  Atomic mode: into every tile its taps reach;
// or, with AE (every warp step of every window starts at its event, and the
// forward sorted the source records by the tiles their events' taps reach),
// one record per source record at the source record's own index: the
// records then come out in bin order, with no count and no scan.
template <int RM, int NT, bool DET, int FM, bool AE>
__global__ __launch_bounds__(NT, 3) void bwd_sweep_kernel(
    const WinMeta* __restrict__ meta, int nw, const int* __restrict__ win_of, const SrcRec* __restrict__ src,
    const uint32_t* __restrict__ start_src, const float* __restrict__ rho,
    const float* __restrict__ ego, const Motion* __restrict__ mtab,
    const double2* __restrict__ img_base, const StateHeader* __restrict__ hdrs,
    const uint32_t* __restrict__ offs, const uint32_t* __restrict__ start,
    GradRec* __restrict__ rec)
{
    extern __shared__ uint32_t lh[];
    const int64_t blk = xcd_block();
    const int w = win_of[blk];
    const WinParams& P = meta[w].P;
    const TileGeom G = meta[w].G;
    const int64_t lb = blk - meta[w].blk_off;
    const SrcRange sr = src_range<DET>(meta[w], hdrs[w], src, start_src);
    const int64_t nv = sr.n;
    const SrcRec* wsrc = sr.p;
    if (!AE) {
        const uint32_t* row = offs + meta[w].hist_off + lb * G.nbins_b;
        for (int i = threadIdx.x; i < G.nbins_b; i += blockDim.x)
            lh[i] = DET ? row[i] : row[i] + start[meta[w].bbin_off + i];
    }
    __syncthreads();
    __shared__ RefTable rt;
    load_ref_table(P, hdrs + w, rt);
    __shared__ MotionTable mt;
    const Flows<FM> u = make_flows_tab<FM>(P, rho + meta[w].pix_off, ego + 6 * meta[w].ego_off,
                                           mtab + meta[w].ego_off, &mt);
    __syncthreads();
    const double2* img = img_base + meta[w].img_off;
    const bool split = FM != 0 && P.F > 1;    // one record per first step (see for_each_sample)

    auto emit = [&](double X, double Y, double gx, double gy, int set) {
        GradRec q;
        q.X = X;
        q.Y = Y;
        q.gx = gx;
        q.gy = gy;
        const Taps tp = make_taps(P, X, Y);
        if (DET) {
            store_nt(rec + stable_slot(lh, set * G.ntiles + tile_index(G, tp)), q);
        } else {
            for_each_reached(tiles_reached(G, tp) + (uint32_t)(set * G.ntiles), G.ntx,
                             [&](int b) { store_nt(rec + atomicAdd(&lh[b], 1u), q); });
        }
    };

    // (the loop runs until the window's source records are done: with AE a
    // window has up to four per valid event, more than the block geometry's
    // events per lane)
    const int64_t stride = (int64_t)G.nblocks * NT;
    // AE: the record of source record i (its event's dt * adjoint; the
    // position is the source record's)
    double2* const arec = reinterpret_cast<double2*>(rec) + (wsrc - src);
    SrcRec qn;
    int64_t i = (int64_t)lb * NT + threadIdx.x;
    if (i < nv) qn = load_nt(wsrc + i);
    for (; i < nv; i += stride) {
        const SrcRec q = qn;
        if (i + stride < nv) qn = load_nt(wsrc + i + stride);
        double vx[RM], vy[RM];
        Visits v;
        const double x0 = q.x0, y0 = q.y0, tk = fabsf(q.ts);
        if (!warp_visits_v<RM, FM>(P, u, rt, x0, y0, tk, v, [&](int j, double X, double Y, int) {
                vx[j] = X;
                vy[j] = Y;
            })) {
            // (a source record's event is valid: the forward's warp of the
            // same inputs; its slot still gets a record)
            if (AE) store_nt(arec + i, 0.0, 0.0);
            continue;
        }
        const int pol = (__float_as_uint(q.ts) >> 31) ? 1 : 0;
        const double2* planes = img + (size_t)pol * P.HW;
        double g0x = 0.0, g0y = 0.0;     // contributions sampled at the event position
        double Lx = 0.0, Ly = 0.0;
#pragma unroll
        for (int j = RM - 1; j >= 0; --j) {
            if (j < P.R) {
                const VisitStep s = visit_step(P, rt, v, j, tk);
                if (s.step) {
                    if (s.restart) {
                        Lx = 0.0;
                        Ly = 0.0;
                    }
                    const int r = visit_ref(v, j);
                    direct_term(P, planes + (size_t)r * 2 * P.HW, rt.coef[r],
                                1.0 - fabs(rt.t[r] - tk), vx[j], vy[j], Lx, Ly);
                    if (s.first) {
                        if (split) {
                            emit(x0, y0, s.dt * Lx, s.dt * Ly, s.set);
                        } else {
                            g0x += s.dt * Lx;
                            g0y += s.dt * Ly;
                        }
                    } else {
                        const double X = vx[j > 0 ? j - 1 : 0], Y = vy[j > 0 ? j - 1 : 0];
                        emit(X, Y, s.dt * Lx, s.dt * Ly, s.set);
                        double jx, jy;
                        jacobian_t(P, u.at(s.set), X, Y, Lx, Ly, jx, jy);
                        Lx += s.dt * jx;
                        Ly += s.dt * jy;
                    }
                }
            }
        }
        if (AE) store_nt(arec + i, g0x, g0y);
        else if (!split && P.R - (v.eq ? 1 : 0) > 0) emit(x0, y0, g0x, g0y, 0);
    }
}

// Deterministic mode: accumulate dL/du = sum over records of w_tap * (dt *
// adjoint) in LDS in record order; own pixels off the border get d rho and
// their d theta share here, the border and the halo go to buffers for the
// merge.
// (the accumulation splits the cells over kDetAccWaves wavefronts as in
// fwd_tile_det_kernel; the output and its reduction run on the first 256
// threads)
template <bool EXACT>
__global__ __launch_bounds__(64 * kDetAccWaves) void bwd_tile_det_kernel(
    const WinMeta* __restrict__ meta, int nw, const int* __restrict__ win_of, const GradRec* __restrict__ rec,
    const uint32_t* __restrict__ start, const float* __restrict__ rho,
    const float* __restrict__ ego, const float* __restrict__ grad_loss,
    float* __restrict__ drho, double2* __restrict__ halo, double2* __restrict__ border,
    double* __restrict__ part)
{
    __shared__ double2 lds[TLW * TLH];
    __shared__ double red[16 * 6];
    const int64_t gtile = blockIdx.x;       // backward bin: (flow set, tile) of a window
    const int w = win_of[gtile];
    const WinParams& P = meta[w].P;
    const TileGeom G = meta[w].G;
    const int lbin = (int)(gtile - meta[w].bbin_off);
    const int set = lbin / G.ntiles, tile = lbin - set * G.ntiles;
    const int ty = tile / G.ntx, tx = tile - ty * G.ntx;
    const int xo = tx * TW, yo = ty * TH;
    const uint32_t s0 = start[gtile], s1 = start[gtile + 1];
    if (s0 == s1) {
        // no records: dL/du is zero on the tile; write its interior d rho and
        // zero d theta shares (the merge writes column 0 and row 0, and reads
        // border values and halos of occupied bins only)
        float* drho_w = drho + meta[w].pix_off + (size_t)set * P.HW;
        const float z = (float)((double)grad_loss[w] * 0.0);
        for (int i = threadIdx.x; i < TW * TH; i += blockDim.x) {
            const int lx = i % TW, ly = i / TW;
            const int X = xo + lx, Y = yo + ly;
            if (X >= P.W || Y >= P.H || lx == 0 || ly == 0) continue;
            drho_w[Y * P.W + X] = z;
        }
        if (threadIdx.x < 6) part[gtile * 12 + threadIdx.x] = 0.0;
        return;
    }
    for (int i = threadIdx.x; i < TLW * TLH; i += blockDim.x) lds[i] = make_double2(0.0, 0.0);
    __syncthreads();
    {
        const int wave = (int)(threadIdx.x >> 6);
        for (uint32_t b0 = s0; b0 < s1; b0 += 64) {
            const uint32_t i = b0 + __lane_id();
            const bool live = i < s1;
            GradRec q;
            if (live) q = rec[i];
            else q.X = q.Y = (double)xo, q.gx = q.gy = 0.0;
            const Taps tp = make_taps(P, q.X, q.Y);
            const int lx = tp.x0 - xo, ly = tp.y0 - yo;
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                const double wt = tap_w(tp, c);
                const int key = (ly + (c >> 1)) * TLW + lx + (c & 1);
                const bool act = live && tap_in(tp, c) && wt != 0.0 && key % kDetAccWaves == wave;
                ordered_add(lds, act, key, wt * q.gx, wt * q.gy);
            }
        }
    }
    __syncthreads();
    const float* ego_s = ego + 6 * (meta[w].ego_off + set);
    const Motion m = load_motion(P, ego_s);
    __shared__ MotionXJ mx[1];      // used by the exact model only
    if (EXACT) {
        if (threadIdx.x == 0) mx[0] = load_motion_xj(ego_s);
        __syncthreads();
    }
    const float* rho_w = rho + meta[w].pix_off + (size_t)set * P.HW;
    float* drho_w = drho + meta[w].pix_off + (size_t)set * P.HW;
    const double gl = (double)grad_loss[w];
    double dth[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    for (int i = threadIdx.x; i < TW * TH && threadIdx.x < 256; i += 256) {
        const int lx = i % TW, ly = i / TW;
        const int X = xo + lx, Y = yo + ly;
        if (X >= P.W || Y >= P.H) continue;
        const double2 g = lds[ly * TLW + lx];
        if (lx == 0 || ly == 0) {
            border[gtile * NBORDER + (lx == 0 ? ly : TH + lx - 1)] = g;
            continue;
        }
        const int pix = Y * P.W + X;
        if constexpr (EXACT) {
            double d = 0.0;
            if (g.x != 0.0 || g.y != 0.0) d = chain_exact(P, mx[0], X, Y, (double)rho_w[pix], g.x, g.y, dth);
            drho_w[pix] = (float)(gl * d);
            continue;
        }
        double Ax, Ay, Bx, By;
        flow_parts(P, m, X, Y, Ax, Ay, Bx, By);
        drho_w[pix] = (float)(gl * (g.x * Bx + g.y * By));
        if (g.x != 0.0 || g.y != 0.0) dtheta_at_pixel(P, X, Y, (double)rho_w[pix], g.x, g.y, dth);
    }
    double2* hb = halo + gtile * NHALO;
    for (int j = threadIdx.x; j < NHALO; j += blockDim.x) {
        const int idx = (j <= TH) ? j * TLW + TW : TH * TLW + (j - (TH + 1));
        hb[j] = lds[idx];
    }
    block_sum_n(dth, red, 256 / 64);
    if (threadIdx.x == 0)
#pragma unroll
        for (int c = 0; c < 6; ++c) part[gtile * 12 + c] = dth[c];
}

// Atomic mode: one workgroup per backward bin (flow set, tile of a window)
// owns the tile's TWX x THX pixels.  Its records are every sampling position
// whose taps reach the tile (with AE, its source bin's records, indexed like
// the source records); it accumulates dL/du at the taps inside the tile in
// LDS, then writes d rho of every pixel and reduces the tile's d theta share.
// No halo, no merge.
// Partial d theta per backward bin in the atomic mode: six per wavefront of
// the tile workgroup (four); the finalize adds them.
constexpr int kBwdPartOwn = 24;

template <bool EXACT, bool AE, int TWX, int THX>
__global__ __launch_bounds__(256) void bwd_tile_own_kernel(
    const WinMeta* __restrict__ meta, int nw, const int* __restrict__ win_of, const GradRec* __restrict__ rec,
    const SrcRec* __restrict__ src, const uint32_t* __restrict__ start,
    const uint32_t* __restrict__ start_src,
    const uint32_t* __restrict__ order, const uint32_t* __restrict__ order_n,
    const float* __restrict__ rho,
    const float* __restrict__ ego, const float* __restrict__ grad_loss,
    float* __restrict__ drho, double* __restrict__ part)
{
    constexpr int NT = 256, NPIX = TWX * THX;
    __shared__ double2 lds[NPIX];
    // backward bin: (flow set, tile) of a window, in the order of a
    // heaviest-first list (the source bins' with AE, one per backward bin;
    // else the backward scan's), so that the longest bins are launched first
    const int64_t gtile = order ? (int64_t)occ_entry(order, order_n, blockIdx.x) : (int64_t)blockIdx.x;
    const int w = win_of[gtile];
    const WinParams& P = meta[w].P;
    const TileGeom G = meta[w].G;
    const int lbin = (int)(gtile - meta[w].bbin_off);
    const int set = lbin / G.ntiles, tile = lbin - set * G.ntiles;
    const int ty = tile / G.ntx, tx = tile - ty * G.ntx;
    const int xo = tx * TWX, yo = ty * THX;
    const uint32_t s0 = AE ? start_src[meta[w].sbin_off + tile] : start[gtile];
    const uint32_t s1 = AE ? start_src[meta[w].sbin_off + tile + 1] : start[gtile + 1];
    float* drho_w = drho + meta[w].pix_off + (size_t)set * P.HW;
    const double gl = (double)grad_loss[w];
    if (s0 == s1) {
        // no records: dL/du is zero on the tile
        const float z = (float)(gl * 0.0);
        for (int i = threadIdx.x; i < NPIX; i += NT) {
            const int X = xo + i % TWX, Y = yo + i / TWX;
            if (X < P.W && Y < P.H) drho_w[Y * P.W + X] = z;
        }
        if (threadIdx.x < kBwdPartOwn) part[gtile * kBwdPartOwn + threadIdx.x] = 0.0;
        return;
    }
    // a record: with AE, the event's position from its source record and
    // dt * adjoint from the sweep's 16-byte record at the same index
    const double2* __restrict__ arec = reinterpret_cast<const double2*>(rec);
    auto load_rec = [&](uint32_t i) {
        if constexpr (AE) {
            const SrcRec qs = load_nt(src + i);
            const double2 g = load_nt(arec + i);
            return GradRec{(double)qs.x0, (double)qs.y0, g.x, g.y};
        } else {
            return rec[i];
        }
    };
    // the first round's records, in flight during the clear
    uint32_t i0 = s0 + threadIdx.x;
    GradRec qq[2];
    if (i0 < s1) {
        qq[0] = load_rec(i0);
        qq[1] = load_rec(i0 + NT < s1 ? i0 + NT : i0);
    }
    for (int i = threadIdx.x; i < NPIX; i += NT) lds[i] = make_double2(0.0, 0.0);
    __syncthreads();
    while (i0 < s1) {
        const bool two = i0 + NT < s1;
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            if (u == 1 && !two) break;
            const GradRec q = qq[u];
            const Taps tp = make_taps(P, q.X, q.Y);
            const int lx = tp.x0 - xo, ly = tp.y0 - yo;
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                const int cx = lx + (c & 1), cy = ly + (c >> 1);
                if (!tap_in(tp, c) || (unsigned)cx >= (unsigned)TWX || (unsigned)cy >= (unsigned)THX)
                    continue;
                const double wt = tap_w(tp, c);
                if (wt == 0.0) continue;
                double2* cell = lds + cy * TWX + cx;
                atomicAdd(&cell->x, wt * q.gx);
                atomicAdd(&cell->y, wt * q.gy);
            }
        }
        i0 += 2 * NT;
        if (i0 < s1) {
            qq[0] = load_rec(i0);
            qq[1] = load_rec(i0 + NT < s1 ? i0 + NT : i0);
        }
    }
    __syncthreads();
    const float* ego_s = ego + 6 * (meta[w].ego_off + set);
    const Motion m = load_motion(P, ego_s);
    __shared__ MotionXJ mx[1];      // used by the exact model only
    if (EXACT) {
        if (threadIdx.x == 0) mx[0] = load_motion_xj(ego_s);
        __syncthreads();
    }
    const float* rho_w = rho + meta[w].pix_off + (size_t)set * P.HW;
    double dth[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    for (int i = threadIdx.x; i < NPIX; i += NT) {
        const int X = xo + i % TWX, Y = yo + i / TWX;
        if (X >= P.W || Y >= P.H) continue;
        const double2 g = lds[i];
        const int pix = Y * P.W + X;
        if constexpr (EXACT) {
            double d = 0.0;
            if (g.x != 0.0 || g.y != 0.0) d = chain_exact(P, mx[0], X, Y, (double)rho_w[pix], g.x, g.y, dth);
            drho_w[pix] = (float)(gl * d);
            continue;
        }
        double Ax, Ay, Bx, By;
        flow_parts(P, m, X, Y, Ax, Ay, Bx, By);
        drho_w[pix] = (float)(gl * (g.x * Bx + g.y * By));
        if (g.x != 0.0 || g.y != 0.0) dtheta_at_pixel(P, X, Y, (double)rho_w[pix], g.x, g.y, dth);
    }
    // each wavefront's d theta share (DPP sums, no block reduction)
#pragma unroll
    for (int c = 0; c < 6; ++c) dth[c] = wave_sum_dpp(dth[c]);
    if ((threadIdx.x & 63) == 63)
#pragma unroll
        for (int c = 0; c < 6; ++c) part[gtile * kBwdPartOwn + (threadIdx.x >> 6) * 6 + c] = dth[c];
}

template <bool EXACT>
__global__ __launch_bounds__(64 * kMergeBins) void bwd_merge_kernel(
    const WinMeta* __restrict__ meta, int nw, int64_t nbins, const int* __restrict__ win_of,
    const float* __restrict__ rho, const float* __restrict__ ego, const float* __restrict__ grad_loss,
    const uint32_t* __restrict__ start, float* __restrict__ drho, const double2* __restrict__ halo,
    const double2* __restrict__ border, double* __restrict__ part)
{
    // one wavefront per backward bin (flow set, tile) of a window
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int64_t graw = (int64_t)blockIdx.x * kMergeBins + wv;
    const bool live = graw < nbins;
    const int64_t gtile = live ? graw : nbins - 1;   // a dead wave reads a valid bin, writes nothing
    const int w = win_of[gtile];
    const WinParams& P = meta[w].P;
    const TileGeom G = meta[w].G;
    const int lbin = (int)(gtile - meta[w].bbin_off);
    const int set = lbin / G.ntiles, tile = lbin - set * G.ntiles;
    const int ty = tile / G.ntx, tx = tile - ty * G.ntx;
    const int xo = tx * TW, yo = ty * TH;
    const float* ego_s = ego + 6 * (meta[w].ego_off + set);
    const Motion m = load_motion(P, ego_s);
    __shared__ MotionXJ mx[kMergeBins];      // used by the exact model only
    if (EXACT) {
        if (lane == 0) mx[wv] = load_motion_xj(ego_s);
        __syncthreads();
    }
    if (!live) return;
    const float* rho_w = rho + meta[w].pix_off + (size_t)set * P.HW;
    float* drho_w = drho + meta[w].pix_off + (size_t)set * P.HW;
    const double gl = (double)grad_loss[w];
    double dth[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    // border values and halos exist for occupied bins only (zero otherwise)
    auto occupied = [&](int64_t b) { return start[b] != start[b + 1]; };
    const bool own = occupied(gtile);
    const bool left = tx > 0 && occupied(gtile - 1);
    const bool up = ty > 0 && occupied(gtile - G.ntx);
    const bool upleft = tx > 0 && ty > 0 && occupied(gtile - G.ntx - 1);
    for (int j = lane; j < NBORDER; j += 64) {
        const int lx = j < TH ? 0 : j - TH + 1;
        const int ly = j < TH ? j : 0;
        const int X = xo + lx, Y = yo + ly;
        if (X >= P.W || Y >= P.H) continue;
        double2 g = own ? border[gtile * NBORDER + j] : make_double2(0.0, 0.0);
        if (lx == 0 && left) {
            const double2 h = halo[(gtile - 1) * NHALO + ly];
            g.x += h.x;
            g.y += h.y;
        }
        if (ly == 0 && up) {
            const double2 h = halo[(gtile - G.ntx) * NHALO + TH + 1 + lx];
            g.x += h.x;
            g.y += h.y;
        }
        if (lx == 0 && ly == 0 && upleft) {
            const double2 h = halo[(gtile - G.ntx - 1) * NHALO + TH];
            g.x += h.x;
            g.y += h.y;
        }
        const int pix = Y * P.W + X;
        if constexpr (EXACT) {
            double d = 0.0;
            if (g.x != 0.0 || g.y != 0.0) d = chain_exact(P, mx[wv], X, Y, (double)rho_w[pix], g.x, g.y, dth);
            drho_w[pix] = (float)(gl * d);
            continue;
        }
        double Ax, Ay, Bx, By;
        flow_parts(P, m, X, Y, Ax, Ay, Bx, By);
        drho_w[pix] = (float)(gl * (g.x * Bx + g.y * By));
        if (g.x != 0.0 || g.y != 0.0) dtheta_at_pixel(P, X, Y, (double)rho_w[pix], g.x, g.y, dth);
    }
#pragma unroll
    for (int c = 0; c < 6; ++c) {
        const double v = wave_sum(dth[c]);
        if (lane == 0) part[gtile * 12 + 6 + c] = v;
    }
}

// One block per window: fixed-order sum of its tiles' d theta partials, per
// flow set (the six components through one block reduction, each in
// block_sum's order).
// (pstride doubles per backward bin: groups of six, two in the deterministic
// mode (tile and merge), one per wavefront in the atomic mode)
__global__ __launch_bounds__(256) void bwd_finalize_kernel(const WinMeta* __restrict__ meta,
                                                           const double* __restrict__ part,
                                                           int pstride, int max_F,
                                                           const StateHeader* __restrict__ hdrs,
                                                           const float* __restrict__ grad_loss,
                                                           float* __restrict__ grad_ego)
{
    __shared__ double red[16 * 6];
    // one workgroup per (window, flow set): blockIdx.x = w * max_F + f
    const int w = (int)blockIdx.x / max_F, f = (int)blockIdx.x - w * max_F;
    if (f >= meta[w].P.F) return;
    const int ntiles = meta[w].G.ntiles;
    const int ng = ntiles * (pstride / 6);
    const double gl = (hdrs[w].flags & kHdrSourceRecords) ? (double)grad_loss[w] : (double)NAN;
    {
        const double* pw = part + (meta[w].bbin_off + (int64_t)f * ntiles) * pstride;
        // (each group's six values read together; every sum still adds the
        // groups in order)
        double v[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
        for (int j = threadIdx.x; j < ng; j += blockDim.x) {
            const double* q = pw + (size_t)j * 6;
#pragma unroll
            for (int c = 0; c < 6; ++c) v[c] += q[c];
        }
        block_sum_n(v, red);
        if (threadIdx.x == 0)
#pragma unroll
            for (int c = 0; c < 6; ++c) grad_ego[(meta[w].ego_off + f) * 6 + c] = (float)(gl * v[c]);
    }
}

// Writes one window's metadata (single-window calls pass it by value).
__global__ void store_meta_kernel(WinMeta m, WinMeta* __restrict__ out)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) out[0] = m;
}

// ---------------------------------------------------------------------------
// Host side: geometry, layout, launches
// ---------------------------------------------------------------------------

// Threads of the count / scatter / sweep blocks: one wavefront in the
// deterministic mode (its record order is the lanes' order), else four.
static int bin_threads(bool det) { return det ? 64 : kBinThreads; }

// Blocks a batch's event kernels aim for (PlanTuning::event_blocks, default
// 4096): a few waves of the 256 CUs, so that every block warps several events
// per lane and the next event's loads overlap the current one's gathers.

static int log2_of(int v)
{
    int s = 0;
    while ((1 << s) < v) ++s;
    return s;
}

TileGeom tile_geom(const WinParams& P, int64_t n, bool det, int min_ept, int tw, int th)
{
    TileGeom G;
    G.tw = det ? TW : tw;
    G.th = det ? TH : th;
    G.tws = log2_of(G.tw);
    G.ths = log2_of(G.th);
    G.ntx = (P.W + G.tw - 1) / G.tw;
    G.nty = (P.H + G.th - 1) / G.th;
    G.ntiles = G.ntx * G.nty;
    G.nbins = P.R * G.ntiles;
    G.nbins_b = P.F * G.ntiles;
    G.nbins_s = det ? 0 : G.ntiles;
    // enough blocks to fill the chip, few enough to keep the histogram matrix small
    const int nt = bin_threads(det);
    const int64_t ept = std::max<int64_t>(n / ((int64_t)nt * 1024), min_ept);
    G.ept = (int)std::max<int64_t>(1, std::min<int64_t>(ept, kMaxEventsPerThread));
    const int64_t per_block = (int64_t)nt * G.ept;
    G.nblocks = (int)std::max<int64_t>(1, (n + per_block - 1) / per_block);
    return G;
}

// The backward of every window samples the flow at its events only (one flow
// set, and references {0, 1} or a single one): every warp step starts at the
// event.
static bool samples_at_events(const WinParams& P)
{
    return P.F == 1 && (P.R == 1 || (P.R == 2 && P.refs[0] == 0.0 && P.refs[1] == 1.0));
}

bool tiled_supported(const WinParams& P, int64_t n, bool det)
{
    const TileGeom G = tile_geom(P, n, det, 1, TW, TH);
    // record slots are 32-bit: up to four per position in the atomic mode
    return G.nbins + G.nbins_s <= kMaxBins && G.nbins_b <= kMaxBins &&
           n * (int64_t)(P.R + 1) < ((int64_t)1 << 29);
}

BatchPlanHost plan_batch(const WinParams* params, const int64_t* n_events, int nw, bool det,
                         const PlanTuning& tune)
{
    BatchPlanHost B;
    B.nw = nw;
    B.det = det;
    B.tile_threads = det ? kTileThreadsDet : tune.tile_threads;
    const int64_t target_blocks = tune.event_blocks;
    // the tile size (atomic mode): the tuning's, unless a window would then
    // need more bins than the LDS histograms hold
    B.tile_w = det ? TW : tune.tile_w;
    B.tile_h = det ? TH : tune.tile_h;
    for (int w = 0; w < nw && !det; ++w) {
        const TileGeom g = tile_geom(params[w], n_events[w], false, 1, B.tile_w, B.tile_h);
        if (g.nbins + g.nbins_s > kMaxBins || g.nbins_b > kMaxBins) {
            B.tile_w = TW;
            B.tile_h = TH;
            break;
        }
    }
    B.meta.resize(nw);
    int64_t ev = 0, pix = 0, sets = 0, img = 0, hist = 0, csum = 0, bin = 0, bbin = 0, sbin = 0;
    int64_t blk = 0, cf = 0, cb = 0, recs = 0;
    B.max_R = 1;
    B.max_F = 1;
    B.max_lds_bins = 1;
    B.at_events = !det;
    // Events per lane from the batch's size (the atomic mode only: the
    // deterministic mode's block partition, and with it its operation order,
    // depends on the window alone).
    int64_t total = 0;
    for (int w = 0; w < nw; ++w) total += n_events[w];
    const int nt = bin_threads(det);
    const int min_ept = det ? 1
                            : (int)std::min<int64_t>(
                                  kMaxEventsPerThread,
                                  std::max<int64_t>(1, (total + nt * target_blocks - 1) /
                                                           (nt * target_blocks)));
    for (int w = 0; w < nw; ++w) {
        WinMeta& M = B.meta[w];
        std::memset(&M, 0, sizeof M);
        M.P = params[w];
        M.G = tile_geom(M.P, n_events[w], det, min_ept, B.tile_w, B.tile_h);
        M.nchunks = (M.G.nblocks + kScanChunk - 1) / kScanChunk;
        M.ev_off = ev;
        M.n = n_events[w];
        M.pix_off = pix;
        M.ego_off = sets;
        M.img_off = img;
        M.hist_off = hist;
        M.csum_off = csum;
        M.bin_off = bin;
        M.bbin_off = bbin;
        M.sbin_off = sbin;
        M.blk_off = blk;
        M.cell_off_f = cf;
        M.cell_off_b = cb;
        // forward rows (reference and source bins) and backward rows
        const int64_t row = std::max(M.G.nbins + M.G.nbins_s, M.G.nbins_b);
        ev += M.n;
        pix += (int64_t)M.P.F * M.P.HW;
        sets += M.P.F;
        img += (int64_t)2 * M.P.R * M.P.HW;
        hist += (int64_t)M.G.nblocks * row;
        if (det) csum += (int64_t)M.nchunks * row;
        bin += M.G.nbins;
        bbin += M.G.nbins_b;
        sbin += M.G.nbins_s;
        blk += M.G.nblocks;
        cf += (int64_t)M.nchunks * M.G.nbins;
        cb += (int64_t)M.nchunks * M.G.nbins_b;
        recs += M.n * M.P.R;
        B.max_R = std::max(B.max_R, M.P.R);
        B.max_F = std::max(B.max_F, M.P.F);
        B.model = M.P.model;      // uniform over a batch (checked when the batch is created)
        B.max_lds_bins = std::max(B.max_lds_bins, (int)row);
        if (!samples_at_events(M.P)) B.at_events = false;
    }
    B.n_events = ev;
    B.n_pixels = pix;
    B.n_sets = sets;
    B.img_elems = img;
    B.nbins = bin;
    B.nbins_b = bbin;
    B.nbins_s = sbin;
    B.nblocks = blk;
    B.cells_f = cf;
    B.cells_b = cb;
    B.csum_cells = csum;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off += (bytes + 255) / 256 * 256;
        return o;
    };
    // totals and starts: one segment for the reference (forward) or backward
    // bins, one for the source bins (atomic mode)
    B.seg = std::max(bin, bbin);
    B.ws.hist = take((size_t)hist * sizeof(uint32_t));
    B.ws.csum = take((size_t)csum * sizeof(uint32_t));
    // (then, atomic mode: the counters of the heaviest-first bin lists, and
    // the scan chunks' totals)
    const int64_t nchunks = (std::max(bin, bbin) + kScanChunk8k - 1) / kScanChunk8k +
                            (sbin + kScanChunk8k - 1) / kScanChunk8k;
    B.ws.totals =
        take((size_t)(B.seg + 1 + sbin + 2 * kListCounters + nchunks) * sizeof(uint32_t));
    B.ws.start = take((size_t)(B.seg + 1 + sbin + 1) * sizeof(uint32_t));
    // the occupied forward bins, listed by the scan, and their count
    // and (source bins) all of them, heaviest first, for the backward tiles
    // (the forward's bins, then the backward's in the same list, and the
    // source bins)
    B.ws.occ = take((size_t)(3 * std::max(bin, bbin) + 3 * sbin) * sizeof(uint32_t));
    B.ws.part = take((size_t)std::max(bin * (det ? 4 : kPartOwn), bbin * (det ? 12 : kBwdPartOwn)) *
                     sizeof(double));
    B.ws.halo = take(det ? (size_t)std::max<int64_t>(bin * (NHALO + NBORDER) * 2,
                                                     bbin * (NHALO + NBORDER)) *
                               sizeof(double2)
                         : 0);
    // Record slots (32 bytes each): the deterministic mode writes one record
    // per position; the atomic mode one per tile the position's taps reach,
    // at most four (the capacity is that bound; about 7 % above one record
    // per position is typical at 32 x 32 tiles)
    B.ws.records = take((size_t)recs * (det ? 1 : 4) * std::max(sizeof(SplatRec), sizeof(GradRec)));
    // source records: one per valid event, or (atomic, sampled at the events)
    // one per tile the event's taps reach
    B.ws.src = take((size_t)ev * (B.at_events ? 4 : 1) * sizeof(SrcRec));
    B.ws.valid = take((size_t)ev);
    B.ws.win = take((size_t)(blk + bin + bbin) * sizeof(int));
    B.ws.motion = take((size_t)B.n_sets * sizeof(Motion));
    B.ws.tbin = take((size_t)bin * sizeof(TileBin));
    B.ws.total = off;
    return B;
}

// Compute units of the current device (queried once per device).
static int device_cus()
{
    static int cus[64] = {0};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
    if (cus[dev] == 0) {
        int v = 0;
        if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
            v <= 0)
            v = 256;
        cus[dev] = v;
    }
    return cus[dev];
}

// Workgroups per CU of the atomic mode's forward tile kernel: as many as fit
// at once (every workgroup starts at once; each takes its share of the
// heaviest-first list of occupied bins pass by pass).
static int tile_per_cu(const BatchPlanHost& B)
{
    // C and S of both polarities, the touched bytes, the bin table
    const int64_t lds = 2LL * B.tile_w * B.tile_h * (16 + 1) + kBinTable * (int64_t)sizeof(OwnBin);
    return (int)std::max<int64_t>(1, std::min<int64_t>(160 * 1024 / lds,
                                                       32 / (B.tile_threads / 64)));
}

template <int NTT, int TWX, int THX>
static void launch_fwd_tile_own(const BatchPlanHost& B, const TileBin* tbin, const SplatRec* rec,
                                const uint32_t* start, const uint32_t* occ, const uint32_t* occ_n,
                                double2* img, double* part, hipStream_t s)
{
    // (no more workgroups than bins: a small plan takes fewer CUs or slots)
    const int nc = (int)std::max<int64_t>(1, std::min<int64_t>(device_cus(), B.nbins));
    const int per = (int)std::max<int64_t>(
        1, std::min<int64_t>(tile_per_cu(B), (B.nbins + nc - 1) / nc));
    fwd_tile_own_kernel<NTT, TWX, THX><<<nc * per, NTT, 0, s>>>(tbin, rec, start, occ, occ_n,
                                                                img, part, nc);
}

// The atomic mode's tile sizes (the tuning's choice; 32 x 32 by default).
template <typename F>
static void with_tile(const BatchPlanHost& B, F&& f)
{
    using I64 = std::integral_constant<int, 64>;
    using I32 = std::integral_constant<int, 32>;
    using I16 = std::integral_constant<int, 16>;
    if (B.tile_w == 64 && B.tile_h == 32) f(I64(), I32());
    else if (B.tile_w == 32 && B.tile_h == 16) f(I32(), I16());
    else if (B.tile_w == 16 && B.tile_h == 16) f(I16(), I16());
    else f(I32(), I32());
}

static void launch_window_table(const BatchPlanHost& B, const WinMeta* meta, int* tab,
                                const float* ego, Motion* mtab, StateHeader* hdrs,
                                uint32_t* clear, int64_t nclear, TileBin* tbin, hipStream_t s,
                                double* zero2 = nullptr, int64_t nzero2 = 0)
{
    const int64_t n = B.nblocks + B.nbins + B.nbins_b + B.nw + nclear + nzero2;
    window_table_kernel<<<(int)((n + 255) / 256), 256, 0, s>>>(
        meta, B.nw, B.nblocks, B.nbins, B.nbins_b, tab, ego, mtab, hdrs, clear, nclear, tbin,
        zero2, nzero2);
}

// Pointers into a batch's workspace.
struct WsPtrs {
    uint32_t *hist, *csum, *totals, *totals_src, *start, *start_src;
    uint32_t *occ, *occ_n, *occ_src, *occ_src_n;   // heaviest-first bin lists and counters
    uint32_t* chunk_tot;                           // scan chunks' totals
    double* part;
    double2* halo;
    char* records;
    SrcRec* src;
    uint8_t* valid;
    int* wtab;
    Motion* mtab;
    TileBin* tbin;
};

static WsPtrs ws_ptrs(const BatchPlanHost& B, char* ws)
{
    WsPtrs p;
    p.hist = reinterpret_cast<uint32_t*>(ws + B.ws.hist);
    p.csum = reinterpret_cast<uint32_t*>(ws + B.ws.csum);
    p.totals = reinterpret_cast<uint32_t*>(ws + B.ws.totals);
    p.totals_src = p.totals + B.seg + 1;
    p.start = reinterpret_cast<uint32_t*>(ws + B.ws.start);
    p.start_src = p.start + B.seg + 1;
    p.occ = reinterpret_cast<uint32_t*>(ws + B.ws.occ);
    p.occ_src = p.occ + 3 * std::max(B.nbins, B.nbins_b);
    p.occ_n = p.totals_src + B.nbins_s;
    p.occ_src_n = p.occ_n + kListCounters;
    p.chunk_tot = p.occ_src_n + kListCounters;
    p.part = reinterpret_cast<double*>(ws + B.ws.part);
    p.halo = reinterpret_cast<double2*>(ws + B.ws.halo);
    p.records = ws + B.ws.records;
    p.src = reinterpret_cast<SrcRec*>(ws + B.ws.src);
    p.valid = reinterpret_cast<uint8_t*>(ws + B.ws.valid);
    p.wtab = reinterpret_cast<int*>(ws + B.ws.win);
    p.mtab = reinterpret_cast<Motion*>(ws + B.ws.motion);
    p.tbin = reinterpret_cast<TileBin*>(ws + B.ws.tbin);
    return p;
}

template <int RM, bool DET, int FM>
static hipError_t batch_forward_rm(const BatchPlanHost& B, const WinMeta* meta,
                                   const EventPtrs& ev, const float* rho, const float* ego,
                                   float* loss, double2* img, StateHeader* hdrs, char* ws,
                                   hipStream_t s, Profiler* prof)
{
    const int nw = B.nw;
    const WsPtrs W = ws_ptrs(B, ws);
    SplatRec* rec = reinterpret_cast<SplatRec*>(W.records);
    const int* win_blk = W.wtab;
    const int* win_bin = W.wtab + B.nblocks;
    const size_t lds = (size_t)B.max_lds_bins * sizeof(uint32_t);
    constexpr int NT = DET ? 64 : kBinThreads;
    const int ae = B.at_events ? 1 : 0;
    {
        PhaseScope ph(prof, kPhZero, s);
        if (DET)
            launch_window_table(B, meta, W.wtab, ego, W.mtab, hdrs, W.csum, B.csum_cells, W.tbin, s);
        else
            // (and the partial sums: the tile kernel writes those of occupied bins only)
            launch_window_table(B, meta, W.wtab, ego, W.mtab, hdrs, W.totals,
                                B.seg + 1 + B.nbins_s + 2 * kListCounters, W.tbin, s,
                                W.part, B.nbins * kPartOwn);
    }
    {
        PhaseScope ph(prof, kPhCount, s);
        fwd_count_kernel<RM, NT, FM, DET><<<B.nblocks, NT, lds, s>>>(
            meta, nw, win_blk, ev.x, ev.y, ev.t, rho, ego, W.mtab, W.hist, W.csum, W.totals,
            W.totals_src, ae, hdrs, W.valid);
    }
    {
        PhaseScope ph(prof, kPhScan, s);
        if (DET) {
            const int gc = (int)((B.cells_f + 255) / 256);
            chunk_scan_kernel<<<(int)((B.nbins + 255) / 256), 256, 0, s>>>(meta, win_bin, B.nbins,
                                                                            0, W.csum, W.totals);
            scan_kernel<<<1, 1024, 0, s>>>(W.totals, B.nbins, W.start, nullptr, 0, nullptr);
            offsets_kernel<<<gc, 256, 0, s>>>(meta, nw, B.cells_f, 0, W.hist, W.csum, W.start);
        } else {
            const int64_t nc0 = (B.nbins + kScanChunk8k - 1) / kScanChunk8k;
            const int64_t nc1 = (B.nbins_s + kScanChunk8k - 1) / kScanChunk8k;
            const bool sums = nc0 > kScanChunksMax || nc1 > kScanChunksMax;
            if (sums)
                chunk_sums_kernel<<<(int)(nc0 + nc1), 1024, 0, s>>>(W.totals, B.nbins,
                                                                    W.totals_src, B.nbins_s,
                                                                    W.chunk_tot);
            scan_chunks_kernel<<<(int)(nc0 + nc1), 1024, 0, s>>>(
                W.totals, B.nbins, W.start, W.occ, W.occ_n, W.totals_src, B.nbins_s,
                W.start_src, W.occ_src, W.occ_src_n, sums ? W.chunk_tot : nullptr);
        }
    }
    {
        PhaseScope ph(prof, kPhScatter, s);
        fwd_scatter_kernel<RM, NT, DET, FM><<<B.nblocks, NT, lds, s>>>(
            meta, nw, win_blk, ev.x, ev.y, ev.t, ev.p, rho, ego, W.mtab, W.hist, W.start,
            W.start_src, ae, W.valid, rec, W.src);
    }
    {
        PhaseScope ph(prof, kPhSplat, s);
        if (DET)
            fwd_tile_det_kernel<<<(int)B.nbins, 64 * kDetAccWaves, 0, s>>>(
                W.tbin, rec, W.start, img, W.halo, W.halo + B.nbins * NHALO * 2, W.part);
        else
            with_tile(B, [&](auto twc, auto thc) {
                constexpr int TWX = decltype(twc)::value, THX = decltype(thc)::value;
                if (B.tile_threads == 256)
                    launch_fwd_tile_own<256, TWX, THX>(B, W.tbin, rec, W.start, W.occ, W.occ_n,
                                                       img, W.part, s);
                else
                    launch_fwd_tile_own<512, TWX, THX>(B, W.tbin, rec, W.start, W.occ, W.occ_n,
                                                       img, W.part, s);
            });
    }
    if (DET) {
        PhaseScope ph(prof, kPhReduce, s);
        fwd_merge_kernel<<<(int)((B.nbins + kMergeBins - 1) / kMergeBins), 64 * kMergeBins, 0, s>>>(
            W.tbin, B.nbins, W.start, img, W.halo, W.halo + B.nbins * NHALO * 2, W.part);
    }
    {
        PhaseScope ph(prof, kPhFinalize, s);
        // (the deterministic mode keeps 256 threads and its references in
        // turn: its addition order, which the mirror follows; the atomic
        // mode sums every reference at once, a wavefront each)
        if (DET)
            fwd_finalize_kernel<<<nw, 256, 0, s>>>(meta, W.part, 4, 2, 0, hdrs, loss);
        else
            fwd_finalize_kernel<<<nw, 64 * B.max_R, 0, s>>>(meta, W.part, kPartOwn,
                                                            B.tile_threads / 64, 1, hdrs, loss);
    }
    return hipGetLastError();
}

hipError_t launch_forward_batch(const BatchPlanHost& B, const WinMeta* meta, const EventPtrs& ev,
                                const float* rho, const float* ego, float* loss, double2* img,
                                StateHeader* hdrs, char* ws, hipStream_t s, Profiler* prof)
{
#define CM_FWD_D(RM, FM) (B.det ? batch_forward_rm<RM, true, FM>(B, meta, ev, rho, ego, loss, img, hdrs, ws, s, prof) \
                            : batch_forward_rm<RM, false, FM>(B, meta, ev, rho, ego, loss, img, hdrs, ws, s, prof))
#define CM_FWD(RM) (B.model == 1 ? CM_FWD_D(RM, 2) : B.max_F > 1 ? CM_FWD_D(RM, 1) : CM_FWD_D(RM, 0))
    if (B.max_R <= 2) return CM_FWD(2);
    if (B.max_R <= 4) return CM_FWD(4);
    if (B.max_R <= 8) return CM_FWD(8);
    return CM_FWD(16);
#undef CM_FWD
#undef CM_FWD_D
}

template <int RM, bool DET, int FM>
static hipError_t batch_backward_rm(const BatchPlanHost& B, const WinMeta* meta,
                                    const EventPtrs& ev, const float* rho, const float* ego,
                                    const double2* img, const StateHeader* hdrs,
                                    const float* grad_loss, float* grad_rho, float* grad_ego,
                                    char* ws, hipStream_t s, Profiler* prof)
{
    const int nw = B.nw;
    const WsPtrs W = ws_ptrs(B, ws);
    GradRec* rec = reinterpret_cast<GradRec*>(W.records);
    const int* win_blk = W.wtab;
    const int* win_tile = W.wtab + B.nblocks + B.nbins;
    const size_t lds = (size_t)B.max_lds_bins * sizeof(uint32_t);
    constexpr int NT = DET ? 64 : kBinThreads;
    constexpr bool EX = FM == 2;
    // sampled at the events only: the forward's source bins are the backward's
    const bool ae = !DET && B.at_events;
    {
        PhaseScope ph(prof, kPhGradCount, s);
        // rebuilt rather than taken from the forward: a state the direct
        // forward filled has no tables, and the backward must stay in bounds
        if (DET)
            launch_window_table(B, meta, W.wtab, ego, W.mtab, nullptr, W.csum, B.csum_cells,
                                W.tbin, s);
        else
            // (and, after the backward bins' totals, the counters of their
            // heaviest-first list: forward-only data lies there)
            launch_window_table(B, meta, W.wtab, ego, W.mtab, nullptr, W.totals,
                                ae ? 0 : B.nbins_b + kListCounters, W.tbin, s);
        if (!ae)
            bwd_count_kernel<RM, NT, FM, DET><<<B.nblocks, NT, lds, s>>>(
                meta, nw, win_blk, W.src, W.start_src, rho, ego, W.mtab, hdrs, W.hist, W.csum,
                W.totals);
    }
    if (!ae) {
        PhaseScope ph(prof, kPhGradScan, s);
        if (DET) {
            const int gc = (int)((B.cells_b + 255) / 256);
            chunk_scan_kernel<<<(int)((B.nbins_b + 255) / 256), 256, 0, s>>>(
                meta, win_tile, B.nbins_b, 1, W.csum, W.totals);
            scan_kernel<<<1, 1024, 0, s>>>(W.totals, B.nbins_b, W.start, nullptr, 0, nullptr);
            offsets_kernel<<<gc, 256, 0, s>>>(meta, nw, B.cells_b, 1, W.hist, W.csum, W.start);
        } else {
            // one array, its list holding the empty bins too (one workgroup per bin)
            const int64_t nc = (B.nbins_b + kScanChunk8k - 1) / kScanChunk8k;
            const bool sums = nc > kScanChunksMax;
            if (sums)
                chunk_sums_kernel<<<(int)nc, 1024, 0, s>>>(nullptr, 0, W.totals, B.nbins_b,
                                                           W.chunk_tot);
            scan_chunks_kernel<<<(int)nc, 1024, 0, s>>>(
                nullptr, 0, nullptr, nullptr, nullptr, W.totals, B.nbins_b, W.start, W.occ,
                W.totals + B.nbins_b, sums ? W.chunk_tot : nullptr);
        }
    }
    {
        PhaseScope ph(prof, kPhAdjoint, s);
        if (ae)
            bwd_sweep_kernel<RM, NT, false, FM, true><<<B.nblocks, NT, 0, s>>>(
                meta, nw, win_blk, W.src, W.start_src, rho, ego, W.mtab, img, hdrs, nullptr,
                nullptr, rec);
        else
            bwd_sweep_kernel<RM, NT, DET, FM, false><<<B.nblocks, NT, lds, s>>>(
                meta, nw, win_blk, W.src, W.start_src, rho, ego, W.mtab, img, hdrs, W.hist,
                W.start, rec);
    }
    {
        PhaseScope ph(prof, kPhGradTile, s);
        if (DET) {
            double2* border = W.halo + B.nbins_b * NHALO;
            bwd_tile_det_kernel<EX><<<(int)B.nbins_b, 64 * kDetAccWaves, 0, s>>>(
                meta, nw, win_tile, rec, W.start, rho, ego, grad_loss, grad_rho, W.halo, border,
                W.part);
            bwd_merge_kernel<EX><<<(int)((B.nbins_b + kMergeBins - 1) / kMergeBins),
                                   64 * kMergeBins, 0, s>>>(meta, nw, B.nbins_b, win_tile, rho,
                                                            ego, grad_loss, W.start, grad_rho,
                                                            W.halo, border, W.part);
        } else {
            with_tile(B, [&](auto twc, auto thc) {
                constexpr int TWX = decltype(twc)::value, THX = decltype(thc)::value;
                if (ae)
                    bwd_tile_own_kernel<EX, true, TWX, THX><<<(int)B.nbins_b, 256, 0, s>>>(
                        meta, nw, win_tile, rec, W.src, W.start, W.start_src, W.occ_src,
                        W.occ_src_n,
                        rho, ego,
                        grad_loss, grad_rho, W.part);
                else
                    bwd_tile_own_kernel<EX, false, TWX, THX><<<(int)B.nbins_b, 256, 0, s>>>(
                        meta, nw, win_tile, rec, W.src, W.start, W.start_src, W.occ,
                        W.totals + B.nbins_b, rho, ego,
                        grad_loss, grad_rho, W.part);
            });
        }
    }
    {
        PhaseScope ph(prof, kPhGradFinalize, s);
        bwd_finalize_kernel<<<nw * B.max_F, 256, 0, s>>>(meta, W.part, DET ? 12 : kBwdPartOwn,
                                                         B.max_F, hdrs, grad_loss, grad_ego);
    }
    return hipGetLastError();
}

hipError_t launch_backward_batch(const BatchPlanHost& B, const WinMeta* meta,
                                 const EventPtrs& ev, const float* rho, const float* ego,
                                 const double2* img, const StateHeader* hdrs,
                                 const float* grad_loss, float* grad_rho, float* grad_ego,
                                 char* ws, hipStream_t s, Profiler* prof)
{
#define CM_BWD_D(RM, FM) (B.det ? batch_backward_rm<RM, true, FM>(B, meta, ev, rho, ego, img, hdrs, grad_loss, grad_rho, grad_ego, ws, s, prof) \
                            : batch_backward_rm<RM, false, FM>(B, meta, ev, rho, ego, img, hdrs, grad_loss, grad_rho, grad_ego, ws, s, prof))
#define CM_BWD(RM) (B.model == 1 ? CM_BWD_D(RM, 2) : B.max_F > 1 ? CM_BWD_D(RM, 1) : CM_BWD_D(RM, 0))
    if (B.max_R <= 2) return CM_BWD(2);
    if (B.max_R <= 4) return CM_BWD(4);
    if (B.max_R <= 8) return CM_BWD(8);
    return CM_BWD(16);
#undef CM_BWD
#undef CM_BWD_D
}

hipError_t launch_store_meta(const WinMeta& m, WinMeta* out, hipStream_t s)
{
    store_meta_kernel<<<1, 64, 0, s>>>(m, out);
    return hipGetLastError();
}

}  // namespace cm
