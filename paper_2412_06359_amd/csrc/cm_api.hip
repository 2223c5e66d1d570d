// cm_api.hip -- the C ABI declared in include/cmloss.h: argument validation,
// state layout, device selection and kernel launches.
#include <cmath>
#include <cstring>
#include <new>

#include "../../include/cmloss.h"
#include "cm_kernels.hpp"

struct cm_handle_s {
    int device;
    int path;               // CM_PATH_*
    cm::Profiler prof;
};

namespace {

using cm::StateHeader;
using cm::StatePtrs;
using cm::WinParams;

constexpr size_t kAlign = 256;

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

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
    return true;
}

WinParams params_of(const cm_window_desc* d);

// Records a window needs at least before the tiled path pays for its extra
// launches (below it the direct atomic path is faster).
constexpr int64_t kTiledMinRecords = 1 << 17;

struct Layout {
    size_t img_bytes, hdr_off, scratch_off, ws_off, total;
    bool tiled;             // the workspace of the tiled path is present
};

// state = images | header | reduction scratch | tiled-path workspace
Layout layout_of(const cm_window_desc* d, int64_t n)
{
    Layout L;
    L.img_bytes = (size_t)32 * d->n_refs * d->width * d->height;
    L.hdr_off = align_up(L.img_bytes, kAlign);
    L.scratch_off = L.hdr_off + align_up(sizeof(StateHeader), kAlign);
    L.ws_off = L.scratch_off + align_up(cm::kScratchDoubles * sizeof(double), kAlign);
    const WinParams P = params_of(d);
    L.tiled = n > 0 && cm::tiled_supported(P, n);
    L.total = L.ws_off + (L.tiled ? cm::tile_workspace_layout(P, n).total : 0);
    return L;
}

bool choose_tiled(const cm_handle_s* h, const Layout& L, const WinParams& P, int64_t n)
{
    if (!L.tiled || h->path == CM_PATH_DIRECT) return false;
    if (h->path == CM_PATH_TILED) return true;
    return n * (int64_t)P.R >= kTiledMinRecords;
}

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
    return P;
}

StatePtrs state_ptrs(const cm_window_desc* d, int64_t n, void* state)
{
    const Layout L = layout_of(d, n);
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

}  // namespace

extern "C" {

cm_status cm_create(cm_handle* h, int device)
{
    if (!h) return CM_ERR_INVALID_ARG;
    *h = nullptr;
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess) return CM_ERR_HIP;
    if (device < 0 || device >= count) return CM_ERR_INVALID_ARG;
    cm_handle_s* hs = new (std::nothrow) cm_handle_s();
    if (!hs) return CM_ERR_OOM;
    hs->device = device;
    hs->path = CM_PATH_AUTO;
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

cm_status cm_loss_forward(cm_handle h, const cm_window_desc* d, const float* ev_x,
                          const float* ev_y, const float* ev_t, const int8_t* ev_p,
                          int64_t n_events, const float* inv_depth, const float* ego, float* loss,
                          void* state, void* stream)
{
    if (!h || !desc_valid(d) || !events_valid(ev_x, ev_y, ev_t, ev_p, n_events) || !inv_depth ||
        !ego || !loss || !state)
        return CM_ERR_INVALID_ARG;
    if (d->mode != CM_MODE_ATOMIC) return CM_ERR_UNSUPPORTED;
    const Layout L = layout_of(d, n_events);
    const WinParams P = params_of(d);
    if (h->path == CM_PATH_TILED && !L.tiled && n_events > 0) return CM_ERR_UNSUPPORTED;
    DeviceGuard g(h->device);
    if (!g.ok()) return CM_ERR_HIP;
    const cm::EventPtrs ev{ev_x, ev_y, ev_t, ev_p, n_events};
    const StatePtrs sp = state_ptrs(d, n_events, state);
    hipStream_t s = static_cast<hipStream_t>(stream);
    cm::Profiler* prof = h->prof.enabled ? &h->prof : nullptr;
    const hipError_t e =
        choose_tiled(h, L, P, n_events)
            ? cm::launch_forward_tiled(P, ev, inv_depth, ego, loss, sp,
                                       static_cast<char*>(state) + L.ws_off, s, prof)
            : cm::launch_forward(P, ev, inv_depth, ego, loss, sp, s, prof);
    return e == hipSuccess ? CM_OK : CM_ERR_HIP;
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
    if (d->mode != CM_MODE_ATOMIC) return CM_ERR_UNSUPPORTED;
    const Layout L = layout_of(d, n_events);
    const WinParams P = params_of(d);
    if (h->path == CM_PATH_TILED && !L.tiled && n_events > 0) return CM_ERR_UNSUPPORTED;
    DeviceGuard g(h->device);
    if (!g.ok()) return CM_ERR_HIP;
    const cm::EventPtrs ev{ev_x, ev_y, ev_t, ev_p, n_events};
    const StatePtrs sp = state_ptrs(d, n_events, state);
    hipStream_t s = static_cast<hipStream_t>(stream);
    cm::Profiler* prof = h->prof.enabled ? &h->prof : nullptr;
    const hipError_t e =
        choose_tiled(h, L, P, n_events)
            ? cm::launch_backward_tiled(P, ev, inv_depth, ego, sp, grad_loss, grad_inv_depth,
                                        grad_ego, static_cast<char*>(state) + L.ws_off, s, prof)
            : cm::launch_backward(P, ev, inv_depth, ego, sp, grad_loss, grad_inv_depth, grad_ego,
                                  s, prof);
    return e == hipSuccess ? CM_OK : CM_ERR_HIP;
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

}  // extern "C"
