// cm_api.hip -- the C ABI declared in include/cmloss.h: argument validation,
// state layout, path selection, batch plans and hipGraph replay.
#include <cmath>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "../../include/cmloss.h"
#include "cm_kernels.hpp"

struct cm_handle_s {
    int device;
    int path;                               // CM_PATH_*
    cm::PlanTuning tune;                    // batch plans' launch shape (atomic mode)
    int64_t tiled_min_records = 1 << 17;    // CM_PATH_AUTO crossover for single windows
    cm::Profiler prof;
    void* scratch = nullptr;                // this device's address of `scratch` (below)
};

// Scratch of cm_loss_forward_noalloc: one window's whole forward state
// (images, sums, reduction partials, metadata, tiled workspace) lives in this
// file-scope device array, so that call allocates nothing.  Each device the
// library runs on holds its own copy, at its own address, until the process
// ends.  Host code never passes the array's name to a kernel or a copy (on
// the host it is only a stand-in for the device symbol): it uses the address
// hipGetSymbolAddress returned for the device, kept per device below.
static __device__ __align__(256) unsigned char scratch[CM_NOALLOC_MAX_STATE_BYTES];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};  // per-device address of `scratch`, set once

// Looks up (once per device) the device address of `scratch` on `device`,
// which must be the current device.
hipError_t scratch_address(int device, void** out)
{
    *out = nullptr;
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        g_scratch_ptr[device] = p;
    }
    *out = g_scratch_ptr[device];
    return hipSuccess;
}

}  // namespace

namespace {

using cm::BatchPlanHost;
using cm::StateHeader;
using cm::StatePtrs;
using cm::WinMeta;
using cm::WinParams;

constexpr size_t kAlign = 256;

// Records a window needs at least before the tiled path pays for its extra
// launches (below it the direct atomic path is faster).
constexpr int64_t kTiledMinRecords = 1 << 17;   // default tiled_min_records

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

// Segments between consecutive knots {0, 1} U refs (refs validated first).
int n_segments(const cm_window_desc* d)
{
    int nk = d->n_refs;
    if (d->refs[0] > 0.f) ++nk;
    if (d->refs[d->n_refs - 1] < 1.f) ++nk;
    return nk - 1;
}

bool desc_valid(const cm_window_desc* d)
{
    if (!d) return false;
    if (d->width <= 0 || d->height <= 0) return false;
    if ((int64_t)d->width * d->height > (1LL << 28)) return false;
    if (!(std::isfinite(d->fx) && std::isfinite(d->fy) && d->fx > 0.f && d->fy > 0.f)) return false;
    if (!(std::isfinite(d->cx) && std::isfinite(d->cy))) return false;
    if (d->n_refs < 1 || d->n_refs > CM_MAX_REFS) return false;
    for (int r = 0; r < d->n_refs; ++r) {
        if (!(d->refs[r] >= 0.f && d->refs[r] <= 1.f)) return false;
        if (r > 0 && !(d->refs[r] > d->refs[r - 1])) return false;
    }
    if (d->mode != CM_MODE_ATOMIC && d->mode != CM_MODE_DETERMINISTIC) return false;
    if (!(std::isfinite(d->eps) && d->eps > 0.f)) return false;
    if (d->n_flows != 0 && d->n_flows != 1 && d->n_flows != n_segments(d)) return false;
    if (d->flow_model != CM_FLOW_FIRST_ORDER && d->flow_model != CM_FLOW_EXACT) return false;
    return true;
}

// Flow sets of a window: 1 (n_flows 0 or 1) or one per segment.
int flows_of(const cm_window_desc* d) { return d->n_flows > 1 ? d->n_flows : 1; }

WinParams params_of(const cm_window_desc* d)
{
    WinParams P;
    std::memset(&P, 0, sizeof P);
    P.W = d->width;
    P.H = d->height;
    P.R = d->n_refs;
    P.HW = d->width * d->height;
    P.cx = d->cx;
    P.cy = d->cy;
    P.fx = d->fx;
    P.fy = d->fy;
    P.inv_fx = 1.0 / P.fx;
    P.inv_fy = 1.0 / P.fy;
    P.fx_over_fy = P.fx / P.fy;
    P.fy_over_fx = P.fy / P.fx;
    P.xmax = (double)(d->width - 1);
    P.ymax = (double)(d->height - 1);
    P.eps = d->eps;
    P.two_over_R = 2.0 / (double)d->n_refs;
    for (int r = 0; r < d->n_refs; ++r) P.refs[r] = d->refs[r];
    // Flow set of the step into reference r: forward steps cross the segment
    // that ends at r's knot, backward steps the one that starts there.
    P.F = flows_of(d);
    P.model = d->flow_model == CM_FLOW_EXACT ? 1 : 0;
    const int k0 = d->refs[0] > 0.f ? 1 : 0;      // knot index of reference 0
    for (int r = 0; r < d->n_refs; ++r) {
        // (a forward step into the first knot or a backward step into the
        // last cannot happen; the clamp only keeps those entries in range)
        P.sf[r] = (int8_t)(P.F > 1 ? std::max(0, k0 + r - 1) : 0);
        P.sb[r] = (int8_t)(P.F > 1 ? std::min(P.F - 1, k0 + r) : 0);
    }
    return P;
}

// Single-window state = images | header | reduction scratch | metadata |
// tiled-path workspace (present where the tiled path applies).
struct Layout {
    size_t img_bytes, hdr_off, scratch_off, meta_off, ws_off, total;
    bool tiled;
};

Layout layout_of(const cm_window_desc* d, int64_t n)
{
    Layout L;
    L.img_bytes = (size_t)32 * d->n_refs * d->width * d->height;
    L.hdr_off = align_up(L.img_bytes, kAlign);
    L.scratch_off = L.hdr_off + align_up(sizeof(StateHeader), kAlign);
    L.meta_off = L.scratch_off + align_up(cm::scratch_doubles(flows_of(d)) * sizeof(double), kAlign);
    L.ws_off = L.meta_off + align_up(sizeof(WinMeta), kAlign);
    const WinParams P = params_of(d);
    L.tiled = n > 0 && cm::tiled_supported(P, n, d->mode == CM_MODE_DETERMINISTIC);
    L.total = L.ws_off +
              (L.tiled ? cm::plan_batch(&P, &n, 1, d->mode == CM_MODE_DETERMINISTIC).ws.total : 0);
    return L;
}

// The deterministic mode always takes the tiled path (its record order and
// accumulation order are fixed); windows it cannot take are rejected.
bool choose_tiled(const cm_handle_s* h, const cm_window_desc* d, const Layout& L,
                  const WinParams& P, int64_t n)
{
    if (!L.tiled) return false;
    if (d->mode == CM_MODE_DETERMINISTIC) return true;
    if (h->path == CM_PATH_DIRECT) return false;
    if (h->path == CM_PATH_TILED) return true;
    return n * (int64_t)P.R >= h->tiled_min_records;
}

StatePtrs state_ptrs(const Layout& L, void* state)
{
    char* base = static_cast<char*>(state);
    StatePtrs s;
    s.img = reinterpret_cast<double*>(base);
    s.hdr = reinterpret_cast<StateHeader*>(base + L.hdr_off);
    s.scratch = reinterpret_cast<double*>(base + L.scratch_off);
    s.zero_floats = (L.hdr_off + sizeof(StateHeader)) / sizeof(float);
    return s;
}

bool events_valid(const float* x, const float* y, const float* t, const int8_t* p, int64_t n)
{
    if (n < 0) return false;
    if (n > 0 && (!x || !y || !t || !p)) return false;
    return true;
}

// Makes the handle's device current for the duration of a call.
class DeviceGuard {
public:
    explicit DeviceGuard(int dev) : prev_(-1), ok_(true)
    {
        if (hipGetDevice(&prev_) != hipSuccess) { ok_ = false; return; }
        if (prev_ != dev && hipSetDevice(dev) != hipSuccess) ok_ = false;
    }
    ~DeviceGuard()
    {
        int cur = -1;
        if (prev_ >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev_) (void)hipSetDevice(prev_);
    }
    bool ok() const { return ok_; }

private:
    int prev_;
    bool ok_;
};

cm_status status_of(hipError_t e) { return e == hipSuccess ? CM_OK : CM_ERR_HIP; }

}  // namespace

// A batch plan: per-window metadata, the state layout, and (with graphs) the
// hipGraphs of the forward and backward launch sequences.  Without graphs the
// plan owns no device memory: each call copies the metadata into the caller's
// state buffer on the call's stream, so creating and destroying plans never
// synchronises the device.  With graphs the metadata gets a device copy of its
// own (captured graphs cannot copy from pageable host memory).
struct cm_batch_s {
    cm_handle h = nullptr;
    BatchPlanHost B;
    std::vector<int64_t> ev_offsets, pix_offsets, set_offsets;
    WinMeta* d_meta = nullptr;
    size_t img_off = 0, hdr_off = 0, meta_off = 0, ws_off = 0, total = 0;
    bool use_graph = false;
    hipStream_t capture = nullptr;
    struct Graph {
        hipGraphExec_t exec = nullptr;
        std::vector<const void*> key;
    } fwd, bwd;

    ~cm_batch_s()
    {
        if (fwd.exec) (void)hipGraphExecDestroy(fwd.exec);
        if (bwd.exec) (void)hipGraphExecDestroy(bwd.exec);
        if (capture) (void)hipStreamDestroy(capture);
        if (d_meta) (void)hipFree(d_meta);
    }
};

namespace {

// Runs `enqueue(stream, profiler)` directly, or replays a hipGraph captured
// from it on a private stream (recaptured when the buffers change).
template <typename F>
cm_status run_maybe_graph(cm_batch_s* b, cm_batch_s::Graph& g, std::vector<const void*> key,
                          hipStream_t s, void* state, F&& enqueue)
{
    if (!b->use_graph) {
        WinMeta* meta = reinterpret_cast<WinMeta*>(static_cast<char*>(state) + b->meta_off);
        if (hipMemcpyAsync(meta, b->B.meta.data(), sizeof(WinMeta) * b->B.nw,
                           hipMemcpyHostToDevice, s) != hipSuccess)
            return CM_ERR_HIP;
        cm::Profiler* prof = b->h->prof.enabled ? &b->h->prof : nullptr;
        return status_of(enqueue(s, prof, meta));
    }
    if (!g.exec || g.key != key) {
        if (g.exec) {
            (void)hipGraphExecDestroy(g.exec);
            g.exec = nullptr;
        }
        hipError_t e = hipStreamBeginCapture(b->capture, hipStreamCaptureModeThreadLocal);
        if (e != hipSuccess) return CM_ERR_HIP;
        const hipError_t el = enqueue(b->capture, nullptr, b->d_meta);
        hipGraph_t graph = nullptr;
        e = hipStreamEndCapture(b->capture, &graph);
        if (el != hipSuccess || e != hipSuccess) {
            if (graph) (void)hipGraphDestroy(graph);
            return CM_ERR_HIP;
        }
        e = hipGraphInstantiate(&g.exec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (e != hipSuccess) {
            g.exec = nullptr;
            return CM_ERR_HIP;
        }
        g.key = std::move(key);
    }
    return status_of(hipGraphLaunch(g.exec, s));
}

}  // namespace

extern "C" {

cm_status cm_create(cm_handle* h, int device)
{
    if (!h) return CM_ERR_INVALID_ARG;
    *h = nullptr;
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess) return CM_ERR_HIP;
    if (device < 0 || device >= count) return CM_ERR_INVALID_ARG;
    void* scratch_ptr = nullptr;
    {
        DeviceGuard g(device);
        if (!g.ok()) return CM_ERR_HIP;
        if (scratch_address(device, &scratch_ptr) != hipSuccess) return CM_ERR_HIP;
    }
    cm_handle_s* hs = new (std::nothrow) cm_handle_s();
    if (!hs) return CM_ERR_OOM;
    hs->device = device;
    hs->path = CM_PATH_AUTO;
    hs->scratch = scratch_ptr;
    *h = hs;
    return CM_OK;
}

cm_status cm_destroy(cm_handle h)
{
    delete h;
    return CM_OK;
}

const char* cm_status_string(cm_status s)
{
    switch (s) {
    case CM_OK: return "CM_OK";
    case CM_ERR_INVALID_ARG: return "CM_ERR_INVALID_ARG";
    case CM_ERR_OOM: return "CM_ERR_OOM";
    case CM_ERR_HIP: return "CM_ERR_HIP";
    case CM_ERR_UNSUPPORTED: return "CM_ERR_UNSUPPORTED";
    case CM_ERR_BUDGET: return "CM_ERR_BUDGET";
    }
    return "CM_ERR_UNKNOWN";
}

size_t cm_state_bytes(const cm_window_desc* d, int64_t n_events)
{
    if (!desc_valid(d) || n_events < 0) return 0;
    return layout_of(d, n_events).total;
}

cm_status cm_set_path(cm_handle h, int path)
{
    if (!h || path < CM_PATH_AUTO || path > CM_PATH_TILED) return CM_ERR_INVALID_ARG;
    h->path = path;
    return CM_OK;
}

cm_status cm_set_tuning(cm_handle h, const cm_tuning* t)
{
    if (!h || !t) return CM_ERR_INVALID_ARG;
    const int eb = t->event_blocks ? t->event_blocks : 4096;
    const int tt = t->tile_threads ? t->tile_threads : 512;
    const int64_t tm = t->tiled_min_records ? t->tiled_min_records : kTiledMinRecords;
    const int tw = t->tile_w ? t->tile_w : 32;
    const int th = t->tile_h ? t->tile_h : 32;
    const bool tile_ok = (tw == 32 && th == 32) || (tw == 64 && th == 32) ||
                         (tw == 32 && th == 16) || (tw == 16 && th == 16);
    if (eb < 256 || eb > 65536 || (tt != 256 && tt != 512) || tm < 1 || !tile_ok)
        return CM_ERR_INVALID_ARG;
    h->tune.event_blocks = eb;
    h->tune.tile_threads = tt;
    h->tune.tile_w = tw;
    h->tune.tile_h = th;
    h->tiled_min_records = tm;
    return CM_OK;
}

cm_status cm_get_tuning(cm_handle h, cm_tuning* out)
{
    if (!h || !out) return CM_ERR_INVALID_ARG;
    out->event_blocks = h->tune.event_blocks;
    out->tile_threads = h->tune.tile_threads;
    out->tiled_min_records = h->tiled_min_records;
    out->tile_w = h->tune.tile_w;
    out->tile_h = h->tune.tile_h;
    return CM_OK;
}

}  // extern "C"

namespace {

// The forward of one window on `state` (a caller buffer, or this device's
// `scratch`), with arguments already validated and L = layout_of(d, n).
cm_status forward_on_state(cm_handle h, const cm_window_desc* d, const Layout& L,
                           const float* ev_x, const float* ev_y, const float* ev_t,
                           const int8_t* ev_p, int64_t n_events, const float* inv_depth,
                           const float* ego, float* loss, void* state, hipStream_t s,
                           cm::Profiler* prof)
{
    const WinParams P = params_of(d);
    const cm::EventPtrs ev{ev_x, ev_y, ev_t, ev_p, n_events};
    const StatePtrs sp = state_ptrs(L, state);
    if (!choose_tiled(h, d, L, P, n_events))
        return status_of(cm::launch_forward(P, ev, inv_depth, ego, loss, sp, s, prof));
    char* base = static_cast<char*>(state);
    const BatchPlanHost B =
        cm::plan_batch(&P, &n_events, 1, d->mode == CM_MODE_DETERMINISTIC);
    WinMeta* meta = reinterpret_cast<WinMeta*>(base + L.meta_off);
    hipError_t e = cm::launch_store_meta(B.meta[0], meta, s);
    if (e != hipSuccess) return CM_ERR_HIP;
    return status_of(cm::launch_forward_batch(B, meta, ev, inv_depth, ego, loss,
                                              reinterpret_cast<double2*>(sp.img), sp.hdr,
                                              base + L.ws_off, s, prof));
}

}  // namespace

extern "C" {

cm_status cm_loss_forward(cm_handle h, const cm_window_desc* d, const float* ev_x,
                          const float* ev_y, const float* ev_t, const int8_t* ev_p,
                          int64_t n_events, const float* inv_depth, const float* ego, float* loss,
                          void* state, void* stream)
{
    if (!h || !desc_valid(d) || !events_valid(ev_x, ev_y, ev_t, ev_p, n_events) || !inv_depth ||
        !ego || !loss || !state)
        return CM_ERR_INVALID_ARG;
    const Layout L = layout_of(d, n_events);
    if ((h->path == CM_PATH_TILED || d->mode == CM_MODE_DETERMINISTIC) && !L.tiled && n_events > 0)
        return CM_ERR_UNSUPPORTED;
    DeviceGuard g(h->device);
    if (!g.ok()) return CM_ERR_HIP;
    return forward_on_state(h, d, L, ev_x, ev_y, ev_t, ev_p, n_events, inv_depth, ego, loss,
                            state, static_cast<hipStream_t>(stream),
                            h->prof.enabled ? &h->prof : nullptr);
}

cm_status cm_loss_forward_noalloc(cm_handle h, const cm_window_desc* d, const float* ev_x,
                                  const float* ev_y, const float* ev_t, const int8_t* ev_p,
                                  int64_t n_events, const float* inv_depth, const float* ego,
                                  float* loss, void* stream)
{
    if (!h || !desc_valid(d) || !events_valid(ev_x, ev_y, ev_t, ev_p, n_events) || !inv_depth ||
        !ego || !loss)
        return CM_ERR_INVALID_ARG;
    const Layout L = layout_of(d, n_events);
    if (L.total > (size_t)CM_NOALLOC_MAX_STATE_BYTES) return CM_ERR_BUDGET;
    if ((h->path == CM_PATH_TILED || d->mode == CM_MODE_DETERMINISTIC) && !L.tiled && n_events > 0)
        return CM_ERR_UNSUPPORTED;
    if (!h->scratch) return CM_ERR_HIP;
    DeviceGuard g(h->device);
    if (!g.ok()) return CM_ERR_HIP;
    // No profiler: recording its events could create some.
    return forward_on_state(h, d, L, ev_x, ev_y, ev_t, ev_p, n_events, inv_depth, ego, loss,
                            h->scratch, static_cast<hipStream_t>(stream), nullptr);
}

cm_status cm_loss_backward(cm_handle h, const cm_window_desc* d, const float* ev_x,
                           const float* ev_y, const float* ev_t, const int8_t* ev_p,
                           int64_t n_events, const float* inv_depth, const float* ego,
                           void* state, const float* grad_loss, float* grad_inv_depth,
                           float* grad_ego, void* stream)
{
    if (!h || !desc_valid(d) || !events_valid(ev_x, ev_y, ev_t, ev_p, n_events) || !inv_depth ||
        !ego || !state || !grad_loss || !grad_inv_depth || !grad_ego)
        return CM_ERR_INVALID_ARG;
    const Layout L = layout_of(d, n_events);
    const WinParams P = params_of(d);
    if ((h->path == CM_PATH_TILED || d->mode == CM_MODE_DETERMINISTIC) && !L.tiled && n_events > 0)
        return CM_ERR_UNSUPPORTED;
    DeviceGuard g(h->device);
    if (!g.ok()) return CM_ERR_HIP;
    const cm::EventPtrs ev{ev_x, ev_y, ev_t, ev_p, n_events};
    const StatePtrs sp = state_ptrs(L, state);
    hipStream_t s = static_cast<hipStream_t>(stream);
    cm::Profiler* prof = h->prof.enabled ? &h->prof : nullptr;
    if (!choose_tiled(h, d, L, P, n_events))
        return status_of(cm::launch_backward(P, ev, inv_depth, ego, sp, grad_loss, grad_inv_depth,
                                             grad_ego, s, prof));
    char* base = static_cast<char*>(state);
    const BatchPlanHost B =
        cm::plan_batch(&P, &n_events, 1, d->mode == CM_MODE_DETERMINISTIC);
    WinMeta* meta = reinterpret_cast<WinMeta*>(base + L.meta_off);
    hipError_t e = cm::launch_store_meta(B.meta[0], meta, s);
    if (e != hipSuccess) return CM_ERR_HIP;
    return status_of(cm::launch_backward_batch(B, meta, ev, inv_depth, ego,
                                               reinterpret_cast<const double2*>(sp.img), sp.hdr,
                                               grad_loss, grad_inv_depth, grad_ego,
                                               base + L.ws_off, s, prof));
}

cm_status cm_state_diagnostics(const cm_window_desc* d, const void* state, double* out,
                               void* stream)
{
    if (!desc_valid(d) || !state || !out) return CM_ERR_INVALID_ARG;
    const Layout L = layout_of(d, 0);
    StateHeader hdr;
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (hipMemcpyAsync(&hdr, static_cast<const char*>(state) + L.hdr_off, sizeof hdr,
                       hipMemcpyDeviceToHost, s) != hipSuccess)
        return CM_ERR_HIP;
    if (hipStreamSynchronize(s) != hipSuccess) return CM_ERR_HIP;
    out[0] = hdr.loss;
    out[1] = (double)hdr.n_valid;
    for (int r = 0; r < d->n_refs; ++r) {
        out[2 + r] = hdr.num[r];
        out[2 + d->n_refs + r] = hdr.nact[r];
    }
    return CM_OK;
}

cm_status cm_profile_enable(cm_handle h, int enable)
{
    if (!h) return CM_ERR_INVALID_ARG;
    h->prof.enabled = enable != 0;
    return CM_OK;
}

cm_status cm_profile_read(cm_handle h, double* ms, int64_t* count)
{
    if (!h || !ms || !count) return CM_ERR_INVALID_ARG;
    DeviceGuard g(h->device);
    if (!g.ok()) return CM_ERR_HIP;
    return h->prof.read(ms, count, CM_N_PHASES) == hipSuccess ? CM_OK : CM_ERR_HIP;
}

// ---------------------------------------------------------------------------
// Batches
// ---------------------------------------------------------------------------

cm_status cm_batch_create(cm_handle h, int32_t n_windows, const cm_window_desc* descs,
                          const int64_t* n_events, cm_batch* out)
{
    if (!out) return CM_ERR_INVALID_ARG;
    *out = nullptr;
    if (!h || n_windows < 1 || !descs || !n_events) return CM_ERR_INVALID_ARG;
    std::vector<WinParams> params(n_windows);
    int64_t total_records = 0;
    for (int w = 0; w < n_windows; ++w) {
        if (!desc_valid(&descs[w]) || n_events[w] < 0) return CM_ERR_INVALID_ARG;
        if (descs[w].mode != descs[0].mode) return CM_ERR_INVALID_ARG;
        if (descs[w].flow_model != descs[0].flow_model) return CM_ERR_INVALID_ARG;
        params[w] = params_of(&descs[w]);
        if (!cm::tiled_supported(params[w], n_events[w], descs[0].mode == CM_MODE_DETERMINISTIC))
            return CM_ERR_UNSUPPORTED;
        total_records += n_events[w] * (int64_t)(params[w].R + 1);
    }
    // record slots are 32-bit; the atomic mode reserves up to four per position
    if (total_records * (descs[0].mode == CM_MODE_DETERMINISTIC ? 1 : 4) >= ((int64_t)1 << 31))
        return CM_ERR_UNSUPPORTED;
    DeviceGuard g(h->device);
    if (!g.ok()) return CM_ERR_HIP;
    cm_batch_s* b = new (std::nothrow) cm_batch_s();
    if (!b) return CM_ERR_OOM;
    b->h = h;
    b->B = cm::plan_batch(params.data(), n_events, n_windows,
                          descs[0].mode == CM_MODE_DETERMINISTIC, h->tune);
    b->ev_offsets.resize(n_windows + 1);
    b->pix_offsets.resize(n_windows + 1);
    b->set_offsets.resize(n_windows + 1);
    for (int w = 0; w < n_windows; ++w) {
        b->ev_offsets[w] = b->B.meta[w].ev_off;
        b->pix_offsets[w] = b->B.meta[w].pix_off;
        b->set_offsets[w] = b->B.meta[w].ego_off;
    }
    b->ev_offsets[n_windows] = b->B.n_events;
    b->pix_offsets[n_windows] = b->B.n_pixels;
    b->set_offsets[n_windows] = b->B.n_sets;
    b->img_off = 0;
    b->hdr_off = align_up((size_t)b->B.img_elems * 16, kAlign);
    b->meta_off = b->hdr_off + align_up((size_t)n_windows * sizeof(StateHeader), kAlign);
    b->ws_off = b->meta_off + align_up((size_t)n_windows * sizeof(WinMeta), kAlign);
    b->total = b->ws_off + b->B.ws.total;
    *out = b;
    return CM_OK;
}

cm_status cm_batch_destroy(cm_batch b)
{
    if (!b) return CM_OK;
    DeviceGuard g(b->h->device);
    delete b;
    return CM_OK;
}

size_t cm_batch_state_bytes(cm_batch b) { return b ? b->total : 0; }

cm_status cm_batch_offsets(cm_batch b, int64_t* event_offsets, int64_t* pixel_offsets)
{
    if (!b) return CM_ERR_INVALID_ARG;
    const size_t n = b->ev_offsets.size();
    if (event_offsets) std::memcpy(event_offsets, b->ev_offsets.data(), n * sizeof(int64_t));
    if (pixel_offsets) std::memcpy(pixel_offsets, b->pix_offsets.data(), n * sizeof(int64_t));
    return CM_OK;
}

cm_status cm_batch_flow_offsets(cm_batch b, int64_t* set_offsets)
{
    if (!b || !set_offsets) return CM_ERR_INVALID_ARG;
    std::memcpy(set_offsets, b->set_offsets.data(), b->set_offsets.size() * sizeof(int64_t));
    return CM_OK;
}

// The plan's metadata in device memory (allocated and filled once per plan:
// graphs and the geometry-consistency calls read it there).
static cm_status ensure_device_meta(cm_batch_s* b)
{
    if (b->d_meta) return CM_OK;
    DeviceGuard g(b->h->device);
    if (!g.ok()) return CM_ERR_HIP;
    const size_t bytes = sizeof(WinMeta) * b->B.nw;
    WinMeta* p = nullptr;
    if (hipMalloc(&p, bytes) != hipSuccess) return CM_ERR_OOM;
    if (hipMemcpy(p, b->B.meta.data(), bytes, hipMemcpyHostToDevice) != hipSuccess) {
        (void)hipFree(p);
        return CM_ERR_HIP;
    }
    b->d_meta = p;
    return CM_OK;
}

cm_status cm_batch_set_graph(cm_batch b, int enable)
{
    if (!b) return CM_ERR_INVALID_ARG;
    if (enable) {
        const cm_status st = ensure_device_meta(b);
        if (st != CM_OK) return st;
        if (!b->capture) {
            DeviceGuard g(b->h->device);
            if (!g.ok()) return CM_ERR_HIP;
            if (hipStreamCreateWithFlags(&b->capture, hipStreamNonBlocking) != hipSuccess)
                return CM_ERR_HIP;
        }
    }
    b->use_graph = enable != 0;
    return CM_OK;
}

cm_status cm_loss_forward_batched(cm_batch b, const float* ev_x, const float* ev_y,
                                  const float* ev_t, const int8_t* ev_p, const float* inv_depth,
                                  const float* ego, float* loss, void* state, void* stream)
{
    if (!b || !events_valid(ev_x, ev_y, ev_t, ev_p, b->B.n_events) || !inv_depth || !ego ||
        !loss || !state)
        return CM_ERR_INVALID_ARG;
    DeviceGuard g(b->h->device);
    if (!g.ok()) return CM_ERR_HIP;
    char* base = static_cast<char*>(state);
    const cm::EventPtrs ev{ev_x, ev_y, ev_t, ev_p, b->B.n_events};
    double2* img = reinterpret_cast<double2*>(base + b->img_off);
    StateHeader* hdrs = reinterpret_cast<StateHeader*>(base + b->hdr_off);
    char* ws = base + b->ws_off;
    std::vector<const void*> key{ev_x, ev_y, ev_t, ev_p, inv_depth, ego, loss, state};
    return run_maybe_graph(b, b->fwd, std::move(key), static_cast<hipStream_t>(stream), state,
                           [&](hipStream_t s, cm::Profiler* prof, const WinMeta* meta) {
                               return cm::launch_forward_batch(b->B, meta, ev, inv_depth, ego,
                                                               loss, img, hdrs, ws, s, prof);
                           });
}

cm_status cm_loss_backward_batched(cm_batch b, const float* ev_x, const float* ev_y,
                                   const float* ev_t, const int8_t* ev_p, const float* inv_depth,
                                   const float* ego, void* state, const float* grad_loss,
                                   float* grad_inv_depth, float* grad_ego, void* stream)
{
    if (!b || !events_valid(ev_x, ev_y, ev_t, ev_p, b->B.n_events) || !inv_depth || !ego ||
        !state || !grad_loss || !grad_inv_depth || !grad_ego)
        return CM_ERR_INVALID_ARG;
    DeviceGuard g(b->h->device);
    if (!g.ok()) return CM_ERR_HIP;
    char* base = static_cast<char*>(state);
    const cm::EventPtrs ev{ev_x, ev_y, ev_t, ev_p, b->B.n_events};
    const double2* img = reinterpret_cast<const double2*>(base + b->img_off);
    const StateHeader* hdrs = reinterpret_cast<const StateHeader*>(base + b->hdr_off);
    char* ws = base + b->ws_off;
    std::vector<const void*> key{ev_x, ev_y, ev_t, ev_p, inv_depth, ego, state, grad_loss,
                                 grad_inv_depth, grad_ego};
    return run_maybe_graph(b, b->bwd, std::move(key), static_cast<hipStream_t>(stream), state,
                           [&](hipStream_t s, cm::Profiler* prof, const WinMeta* meta) {
                               return cm::launch_backward_batch(b->B, meta, ev, inv_depth, ego,
                                                                img, hdrs, grad_loss,
                                                                grad_inv_depth, grad_ego, ws, s,
                                                                prof);
                           });
}

cm_status cm_batch_diagnostics(cm_batch b, const void* state, double* out, void* stream)
{
    if (!b || !state || !out) return CM_ERR_INVALID_ARG;
    const int nw = b->B.nw;
    std::vector<StateHeader> hdr(nw);
    hipStream_t s = static_cast<hipStream_t>(stream);
    DeviceGuard g(b->h->device);
    if (!g.ok()) return CM_ERR_HIP;
    if (hipMemcpyAsync(hdr.data(), static_cast<const char*>(state) + b->hdr_off,
                       sizeof(StateHeader) * nw, hipMemcpyDeviceToHost, s) != hipSuccess)
        return CM_ERR_HIP;
    if (hipStreamSynchronize(s) != hipSuccess) return CM_ERR_HIP;
    for (int w = 0; w < nw; ++w) {
        out[2 * w] = hdr[w].loss;
        out[2 * w + 1] = (double)hdr[w].n_valid;
    }
    return CM_OK;
}

cm_status cm_batch_active_pixels(cm_batch b, const void* state, double* out, void* stream)
{
    if (!b || !state || !out) return CM_ERR_INVALID_ARG;
    const int nw = b->B.nw;
    std::vector<StateHeader> hdr(nw);
    hipStream_t s = static_cast<hipStream_t>(stream);
    DeviceGuard g(b->h->device);
    if (!g.ok()) return CM_ERR_HIP;
    if (hipMemcpyAsync(hdr.data(), static_cast<const char*>(state) + b->hdr_off,
                       sizeof(StateHeader) * nw, hipMemcpyDeviceToHost, s) != hipSuccess)
        return CM_ERR_HIP;
    if (hipStreamSynchronize(s) != hipSuccess) return CM_ERR_HIP;
    for (int w = 0; w < nw; ++w)
        for (int r = 0; r < CM_MAX_REFS; ++r)
            out[(size_t)w * CM_MAX_REFS + r] = r < b->B.meta[w].P.R ? hdr[w].nact[r] : 0.0;
    return CM_OK;
}

cm_status cm_batch_occupied_image_bytes(cm_batch b, const void* state, double* out, void* stream)
{
    if (!b || !state || !out) return CM_ERR_INVALID_ARG;
    const BatchPlanHost& B = b->B;
    std::vector<uint32_t> start((size_t)B.nbins + 1);
    hipStream_t s = static_cast<hipStream_t>(stream);
    DeviceGuard g(b->h->device);
    if (!g.ok()) return CM_ERR_HIP;
    if (hipMemcpyAsync(start.data(), static_cast<const char*>(state) + b->ws_off + B.ws.start,
                       sizeof(uint32_t) * start.size(), hipMemcpyDeviceToHost, s) != hipSuccess)
        return CM_ERR_HIP;
    if (hipStreamSynchronize(s) != hipSuccess) return CM_ERR_HIP;
    for (int w = 0; w < B.nw; ++w) {
        const WinMeta& M = B.meta[w];
        double bytes = 0.0;
        for (int bin = 0; bin < M.G.nbins; ++bin) {
            const int64_t gb = M.bin_off + bin;
            if (start[gb + 1] == start[gb]) continue;
            const int tile = bin % M.G.ntiles;
            const int tx = tile % M.G.ntx, ty = tile / M.G.ntx;
            const int pw = std::min(M.G.tw, M.P.W - tx * M.G.tw);
            const int ph = std::min(M.G.th, M.P.H - ty * M.G.th);
            bytes += 2.0 * 16.0 * pw * ph;      // C and S, FP64, both polarities
        }
        out[w] = bytes;
    }
    return CM_OK;
}

// ---------------------------------------------------------------------------
// Geometry consistency (Eq. 3) and the full loss (Eq. 4)
// ---------------------------------------------------------------------------

static cm::GeoLayout geo_layout_one(const cm_window_desc* d)
{
    const int F = flows_of(d);
    const int HW = d->width * d->height;
    return cm::geo_layout(1, F, cm::geo_tiles(d->width, d->height), HW, (int64_t)F * HW,
                          d->mode == CM_MODE_DETERMINISTIC);
}

static cm::GeoLayout geo_layout_batch(const cm_batch_s* b)
{
    int max_F = 1, max_HW = 1, max_tiles = 1;
    for (const WinMeta& m : b->B.meta) {
        max_F = std::max(max_F, m.P.F);
        max_HW = std::max(max_HW, m.P.HW);
        max_tiles = std::max(max_tiles, cm::geo_tiles(m.P.W, m.P.H));
    }
    return cm::geo_layout(b->B.nw, max_F, max_tiles, max_HW, b->B.n_pixels, b->B.det);
}

static WinMeta geo_meta_one(const cm_window_desc* d)
{
    WinMeta m;
    std::memset(&m, 0, sizeof m);
    m.P = params_of(d);
    return m;
}

size_t cm_geo_state_bytes(const cm_window_desc* d)
{
    if (!desc_valid(d)) return 0;
    return geo_layout_one(d).total;
}

cm_status cm_geo_forward(cm_handle h, const cm_window_desc* d, const float* inv_depth,
                         const float* ego, float lambda, const float* loss_cm, float* loss_geo,
                         float* loss_total, void* state, void* stream)
{
    if (!h || !desc_valid(d) || !inv_depth || !ego || !loss_geo || !state ||
        !std::isfinite(lambda))
        return CM_ERR_INVALID_ARG;
    DeviceGuard g(h->device);
    if (!g.ok()) return CM_ERR_HIP;
    const cm::GeoLayout L = geo_layout_one(d);
    hipStream_t s = static_cast<hipStream_t>(stream);
    WinMeta* meta = reinterpret_cast<WinMeta*>(static_cast<char*>(state) + L.meta);
    if (cm::launch_store_meta(geo_meta_one(d), meta, s) != hipSuccess) return CM_ERR_HIP;
    return status_of(cm::launch_geo_forward(L, meta, 1, state, inv_depth, ego, lambda, loss_cm,
                                            loss_geo, loss_total, s));
}

cm_status cm_geo_backward(cm_handle h, const cm_window_desc* d, const float* inv_depth,
                          const float* ego, float lambda, void* state, const float* grad_loss,
                          float* grad_inv_depth, float* grad_ego, void* stream)
{
    if (!h || !desc_valid(d) || !inv_depth || !ego || !state || !grad_loss || !grad_inv_depth ||
        !grad_ego || !std::isfinite(lambda))
        return CM_ERR_INVALID_ARG;
    DeviceGuard g(h->device);
    if (!g.ok()) return CM_ERR_HIP;
    const cm::GeoLayout L = geo_layout_one(d);
    hipStream_t s = static_cast<hipStream_t>(stream);
    WinMeta* meta = reinterpret_cast<WinMeta*>(static_cast<char*>(state) + L.meta);
    if (cm::launch_store_meta(geo_meta_one(d), meta, s) != hipSuccess) return CM_ERR_HIP;
    return status_of(cm::launch_geo_backward(L, meta, 1, state, inv_depth, ego, lambda, grad_loss,
                                             grad_inv_depth, grad_ego, s));
}

size_t cm_batch_geo_state_bytes(cm_batch b) { return b ? geo_layout_batch(b).total : 0; }

cm_status cm_geo_forward_batched(cm_batch b, const float* inv_depth, const float* ego,
                                 float lambda, const float* loss_cm, float* loss_geo,
                                 float* loss_total, void* state, void* stream)
{
    if (!b || !inv_depth || !ego || !loss_geo || !state || !std::isfinite(lambda))
        return CM_ERR_INVALID_ARG;
    DeviceGuard g(b->h->device);
    if (!g.ok()) return CM_ERR_HIP;
    const cm::GeoLayout L = geo_layout_batch(b);
    hipStream_t s = static_cast<hipStream_t>(stream);
    const cm_status st = ensure_device_meta(b);
    if (st != CM_OK) return st;
    return status_of(cm::launch_geo_forward(L, b->d_meta, b->B.nw, state, inv_depth, ego, lambda,
                                            loss_cm, loss_geo, loss_total, s));
}

cm_status cm_geo_backward_batched(cm_batch b, const float* inv_depth, const float* ego,
                                  float lambda, void* state, const float* grad_loss,
                                  float* grad_inv_depth, float* grad_ego, void* stream)
{
    if (!b || !inv_depth || !ego || !state || !grad_loss || !grad_inv_depth || !grad_ego ||
        !std::isfinite(lambda))
        return CM_ERR_INVALID_ARG;
    DeviceGuard g(b->h->device);
    if (!g.ok()) return CM_ERR_HIP;
    const cm::GeoLayout L = geo_layout_batch(b);
    hipStream_t s = static_cast<hipStream_t>(stream);
    const cm_status st = ensure_device_meta(b);
    if (st != CM_OK) return st;
    return status_of(cm::launch_geo_backward(L, b->d_meta, b->B.nw, state, inv_depth, ego, lambda,
                                             grad_loss, grad_inv_depth, grad_ego, s));
}

}  // extern "C"
