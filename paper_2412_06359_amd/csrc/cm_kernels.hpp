// cm_kernels.hpp -- internal interface between the C ABI and the kernels.
#pragma once

#include <algorithm>
#include <cstring>
#include <vector>
#include <stdint.h>

#include "cm_device.hpp"

namespace cm {

// Per-window sums written by the forward (device memory, inside `state`).
struct StateHeader {
    double loss;
    unsigned long long n_valid;
    unsigned long long flags;   // kHdrSourceRecords: written by the tiled forward
    double num[kMaxRefs];
    double nact[kMaxRefs];
};

// The tiled forward leaves per-event source records for the tiled backward;
// a state filled by the direct forward has none, and a tiled backward on it
// returns NaN gradients instead of reading them.
constexpr unsigned long long kHdrSourceRecords = 1ull;

constexpr int kReduceBlocks = 256;     // reduce blocks per reference (max)
constexpr int kBackwardBlocks = 4096;  // backward grid (max), grid-stride beyond
// Reduction scratch of the direct path: forward partials per reference and
// block, backward d theta partials per block and flow set.
inline size_t scratch_doubles(int F)
{
    return std::max<size_t>((size_t)kReduceBlocks * kMaxRefs * 2, (size_t)kBackwardBlocks * 6 * F);
}

struct EventPtrs {
    const float* x;
    const float* y;
    const float* t;
    const int8_t* p;
    int64_t n;
};

struct StatePtrs {
    double* img;           // [R][2][H*W][2] FP64
    StateHeader* hdr;
    double* scratch;       // scratch_doubles(F)
    size_t zero_floats;    // floats to clear before a forward (images + header)
};

// Optional per-phase timing: HIP events recorded on the launch stream around
// each kernel (see cm_profile_enable in include/cmloss.h).
class Profiler {
public:
    bool enabled = false;
    void begin(int phase, hipStream_t s)
    {
        Rec r{phase, get(), get()};
        (void)hipEventRecord(r.a, s);
        recs_.push_back(r);
    }
    void end(hipStream_t s) { (void)hipEventRecord(recs_.back().b, s); }
    // Accumulates elapsed ms and counts per phase, then recycles the events.
    hipError_t read(double* ms, int64_t* count, int n_phases)
    {
        for (int i = 0; i < n_phases; ++i) { ms[i] = 0.0; count[i] = 0; }
        hipError_t err = hipSuccess;
        for (const Rec& r : recs_) {
            float t = 0.f;
            hipError_t e = hipEventSynchronize(r.b);
            if (e == hipSuccess) e = hipEventElapsedTime(&t, r.a, r.b);
            if (e != hipSuccess) err = e;
            if (r.phase >= 0 && r.phase < n_phases) { ms[r.phase] += t; count[r.phase] += 1; }
            pool_.push_back(r.a);
            pool_.push_back(r.b);
        }
        recs_.clear();
        return err;
    }
    ~Profiler()
    {
        for (const Rec& r : recs_) { (void)hipEventDestroy(r.a); (void)hipEventDestroy(r.b); }
        for (hipEvent_t e : pool_) (void)hipEventDestroy(e);
    }

private:
    struct Rec { int phase; hipEvent_t a, b; };
    hipEvent_t get()
    {
        if (!pool_.empty()) { hipEvent_t e = pool_.back(); pool_.pop_back(); return e; }
        hipEvent_t e = nullptr;
        (void)hipEventCreate(&e);
        return e;
    }
    std::vector<Rec> recs_;
    std::vector<hipEvent_t> pool_;
};

// Records a phase around the kernels launched in its scope (no-op without a profiler).
struct PhaseScope {
    PhaseScope(Profiler* p, int phase, hipStream_t s) : p_(p), s_(s) { if (p_) p_->begin(phase, s_); }
    ~PhaseScope() { if (p_) p_->end(s_); }
    Profiler* p_;
    hipStream_t s_;
};

enum Phase {
    kPhZero = 0, kPhSplat, kPhReduce, kPhFinalize, kPhGradZero, kPhAdjoint, kPhGradFinalize,
    kPhCount, kPhScan, kPhScatter, kPhGradCount, kPhGradScan, kPhGradTile, kNumPhases
};

// Per-window metadata of the tiled path (device memory).  All offsets are
// into flat arrays shared by the windows of a batch.
struct WinMeta {
    WinParams P;
    TileGeom G;             // forward bins R * ntiles; backward bins F * ntiles
    int nchunks;            // column-scan chunks of this window's count blocks
    int pad_;
    int64_t ev_off, n;      // events [ev_off, ev_off + n) of the flat event arrays
    int64_t pix_off;        // first pixel of rho / d rho (F images of H W each)
    int64_t ego_off;        // first flow set of ego / d ego (6 floats each)
    int64_t img_off;        // first image element (double2) in the state
    int64_t hist_off;       // first histogram cell
    int64_t csum_off;       // first chunk-sum cell
    int64_t bin_off;        // first forward bin
    int64_t bbin_off;       // first backward bin (flow set, tile)
    int64_t sbin_off;       // first source-record bin (atomic mode)
    int64_t blk_off;        // first count / scatter / sweep block
    int64_t cell_off_f;     // first forward chunk cell
    int64_t cell_off_b;     // first backward chunk cell
};

constexpr int kScanChunk = 16;  // histogram rows per chunk of the column scan

// Byte offsets of the tiled path's buffers inside the workspace region.
struct TileWorkspace {
    size_t hist, csum, totals, start, occ, part, halo, records, src, valid, win, motion, tbin, total;
};

// What the forward tile kernel needs of its bin, in one record written with
// the window table: read together with the bin's bounds, it spares the kernel
// the dependent lookups of the bin's window and the window's parameters.
struct TileBin {
    double ref, eps;        // the bin's reference time; the window's eps
    int64_t plane;          // first element of the bin's (reference, positive) image plane
    int W, H;               // sensor
    int xo, yo;             // tile origin
    int ntx, pad;           // tiles per row
};

// Host-side plan of a tiled batch: per-window metadata, totals, workspace layout.
struct BatchPlanHost {
    int nw = 0;
    bool det = false;       // deterministic mode
    std::vector<WinMeta> meta;
    int64_t n_events = 0, n_pixels = 0, n_sets = 0, img_elems = 0;
    int64_t nbins = 0, nbins_b = 0, nbins_s = 0, nblocks = 0, cells_f = 0, cells_b = 0;
    int64_t csum_cells = 0;
    int64_t seg = 0;        // bins of the first totals / start segment: max(nbins, nbins_b)
    int max_R = 1, max_F = 1, max_lds_bins = 1;
    bool at_events = false; // atomic mode, every window samples the flow at its events only
    int model = 0;          // flow model of the batch's windows
    int tile_threads = 512; // forward tile kernel threads (atomic mode)
    int tile_w = 32, tile_h = 32;   // tile size (atomic mode: the tuning's; 32 x 32 otherwise)
    TileWorkspace ws;
};

// Kernels shared by the direct and tiled paths.
__global__ __launch_bounds__(256) void finalize_forward_kernel(WinParams P,
                                                               const double* __restrict__ part,
                                                               int RB, StateHeader* hdr,
                                                               float* __restrict__ loss);
__global__ __launch_bounds__(256) void finalize_backward_kernel(const double* __restrict__ part,
                                                                int nblk, int F,
                                                                const float* __restrict__ grad_loss,
                                                                float* __restrict__ grad_ego);

int reduce_blocks(const WinParams& P);
int backward_blocks(int64_t n);

hipError_t launch_fill_zero(float* p, size_t n_floats, hipStream_t s);
hipError_t launch_forward(const WinParams& P, const EventPtrs& ev, const float* rho,
                          const float* ego, float* loss, const StatePtrs& st, hipStream_t s,
                          Profiler* prof);
hipError_t launch_backward(const WinParams& P, const EventPtrs& ev, const float* rho,
                           const float* ego, const StatePtrs& st, const float* grad_loss,
                           float* grad_rho, float* grad_ego, hipStream_t s, Profiler* prof);

// Tiled (owner-computes) path over one or many windows.  `meta` is the device
// copy of plan.meta; `ws` a device region of plan.ws.total bytes; images of
// window w start at img + meta[w].img_off; hdrs[w] its sums.
bool tiled_supported(const WinParams& P, int64_t n, bool det);
TileGeom tile_geom(const WinParams& P, int64_t n, bool det, int min_ept, int tw, int th);
// Launch shape of a plan (the atomic mode's tunables; see cm_tuning).
struct PlanTuning {
    int event_blocks = 4096;
    int tile_threads = 512;
    int tile_w = 32, tile_h = 32;
};
BatchPlanHost plan_batch(const WinParams* params, const int64_t* n_events, int nw, bool det,
                         const PlanTuning& tune = PlanTuning());
hipError_t launch_store_meta(const WinMeta& m, WinMeta* out, hipStream_t s);
hipError_t launch_forward_batch(const BatchPlanHost& B, const WinMeta* meta, const EventPtrs& ev,
                                const float* rho, const float* ego, float* loss, double2* img,
                                StateHeader* hdrs, char* ws, hipStream_t s, Profiler* prof);
hipError_t launch_backward_batch(const BatchPlanHost& B, const WinMeta* meta,
                                 const EventPtrs& ev, const float* rho, const float* ego,
                                 const double2* img, const StateHeader* hdrs,
                                 const float* grad_loss, float* grad_rho, float* grad_ego,
                                 char* ws, hipStream_t s, Profiler* prof);


// Geometry consistency (Eq. 3) between consecutive flow sets and the full loss
// (Eq. 4).  Per (window, pair) results of a forward, read by the backward.
struct GeoPairSum {
    double mean;            // mean over V of |D_{0->1} - D'_1| / (D_{0->1} + D'_1)
    double count;           // |V|
    double scale;           // fixed-point scale of the deterministic scatter (2^e)
};

// Byte offsets of the geometry-consistency state: window metadata, block
// partials, pair sums, pair poses, fixed-point accumulator (deterministic mode only, one
// 64-bit cell per inverse-depth pixel).
struct GeoLayout {
    int nblk = 1;           // 32 x 32 tiles per (window, pair) in the grid
    int napply = 1;         // pixel blocks per (window, pair) of the deterministic apply pass
    int npm = 1;            // pair slots per window (max F - 1)
    bool det = false;
    int64_t n_acc = 0;
    size_t meta = 0, part = 0, pairs = 0, poses = 0, acc = 0, total = 0;
};
GeoLayout geo_layout(int nw, int max_F, int max_tiles, int max_HW, int64_t n_pixels, bool det);
inline int geo_tiles(int W, int H) { return ((W + 31) / 32) * ((H + 31) / 32); }
// `meta`: the windows' metadata in device memory (the state's copy, or a
// batch plan's device array).
hipError_t launch_geo_forward(const GeoLayout& L, const WinMeta* meta, int nw, void* state,
                              const float* rho, const float* ego, float lambda,
                              const float* loss_cm, float* loss_geo, float* loss_total,
                              hipStream_t s);
hipError_t launch_geo_backward(const GeoLayout& L, const WinMeta* meta, int nw, void* state,
                               const float* rho, const float* ego, float lambda,
                               const float* grad_loss, float* grad_rho, float* grad_ego,
                               hipStream_t s);

}  // namespace cm
