// cm_tiles.hip -- owner-computes tiled splat (forward) and tiled dL/du
// accumulation (backward) for gfx950.
//
// Scattered global floating-point atomics run at about 22 G/s on MI355X
// whatever the array size (one request per distinct cache line), while LDS
// FP64 atomics run at about 1.4 T/s.  So instead of splatting every tap with a
// global atomic, each warped position becomes a record binned by the 32x32
// tile of its tap (x0, y0) (a counting sort: count, scan, scatter), and one
// workgroup per tile accumulates its records in LDS and writes every pixel it
// owns once with plain, coalesced stores.  A record's taps can reach one
// column right of and one row below its tile; that halo goes to a small
// buffer and a merge pass adds it, in a fixed order, into the column 0 / row 0
// of the neighbouring tiles.
//
// Forward:  count -> colsum -> scan -> offsets -> scatter -> tile -> merge
//           -> finalize.  The per-reference sums of Eq. 1 are reduced in the
//           tile (interior pixels) and merge (border pixels) kernels.
// Backward: count -> colsum -> scan -> offsets -> sweep -> tile -> merge
//           -> finalize.  The sweep re-runs each event's warp, gathers the
//           adjoint seeds, runs the reverse sweep and emits one record per
//           flow-sampling position with dt * adjoint; the tile kernels turn
//           the accumulated dL/du into d rho and d theta per pixel.
#include "cm_kernels.hpp"

namespace cm {

// ---------------------------------------------------------------------------
// Counting sort of records into bins
// ---------------------------------------------------------------------------

// Visit the forward records of one event: fn(bin, r) for every reference.
template <int RM, typename F>
__device__ __forceinline__ void for_each_splat(const WinParams& P, const TileGeom& G,
                                               const double (&px)[RM], const double (&py)[RM],
                                               F&& fn)
{
#pragma unroll
    for (int r = 0; r < RM; ++r) {
        if (r < P.R) {
            const Taps t = make_taps(P, px[r], py[r]);
            fn(r * G.ntiles + tile_index(G, t), r);
        }
    }
}

template <int RM>
__global__ __launch_bounds__(kBinThreads) void fwd_count_kernel(
    WinParams P, TileGeom G, const float* __restrict__ ex, const float* __restrict__ ey,
    const float* __restrict__ et, int64_t n, const float* __restrict__ rho,
    const float* __restrict__ ego, uint32_t* __restrict__ hist,
    unsigned long long* __restrict__ n_valid)
{
    const FlowSrc u = flow_src(P, rho, ego);
    extern __shared__ uint32_t lh[];
    __shared__ uint32_t cnt_lds;
    for (int i = threadIdx.x; i < G.nbins; i += blockDim.x) lh[i] = 0;
    if (threadIdx.x == 0) cnt_lds = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * kBinThreads * G.ept;
    uint32_t cnt = 0;
    for (int e = 0; e < G.ept; ++e) {
        const int64_t k = base + (int64_t)e * kBinThreads + threadIdx.x;
        if (k >= n) break;
        double px[RM], py[RM];
        int mb;
        if (!warp_event<RM>(P, u, ex[k], ey[k], et[k], px, py, mb)) continue;
        ++cnt;
        for_each_splat<RM>(P, G, px, py, [&](int bin, int) { atomicAdd(&lh[bin], 1u); });
    }
    if (cnt) atomicAdd(&cnt_lds, cnt);
    __syncthreads();
    uint32_t* row = hist + (size_t)blockIdx.x * G.nbins;
    for (int i = threadIdx.x; i < G.nbins; i += blockDim.x) row[i] = lh[i];
    if (threadIdx.x == 0 && cnt_lds) atomicAdd(n_valid, (unsigned long long)cnt_lds);
}

// Column scan of the block x bin histogram in two levels: blocks are grouped
// in chunks of kScanChunk rows; chunk sums, then a per-bin scan over chunks,
// then the per-block offsets inside each chunk.  Every step is a short loop
// over many parallel threads.
constexpr int kScanChunk = 16;

// csum[c][bin] = sum of hist[b][bin] for b in chunk c
__global__ __launch_bounds__(256) void chunk_sum_kernel(const uint32_t* __restrict__ hist,
                                                        int nblocks, int nbins, int nchunks,
                                                        uint32_t* __restrict__ csum)
{
    const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= (int64_t)nbins * nchunks) return;
    const int c = (int)(id / nbins), bin = (int)(id - (int64_t)c * nbins);
    const int b0 = c * kScanChunk, b1 = min(b0 + kScanChunk, nblocks);
    uint32_t s = 0;
    for (int b = b0; b < b1; ++b) s += hist[(size_t)b * nbins + bin];
    csum[(size_t)c * nbins + bin] = s;
}

// In place: csum[c][bin] <- sum over chunks before c; totals[bin] = column total.
__global__ __launch_bounds__(256) void chunk_scan_kernel(uint32_t* __restrict__ csum, int nbins,
                                                         int nchunks, uint32_t* __restrict__ totals)
{
    const int bin = blockIdx.x * blockDim.x + threadIdx.x;
    if (bin >= nbins) return;
    uint32_t run = 0;
    for (int c = 0; c < nchunks; ++c) {
        const uint32_t v = csum[(size_t)c * nbins + bin];
        csum[(size_t)c * nbins + bin] = run;
        run += v;
    }
    totals[bin] = run;
}

// start[bin] = exclusive prefix sum of totals; start[nbins] = total.  One block.
__global__ __launch_bounds__(1024) void scan_kernel(const uint32_t* __restrict__ totals, int nbins,
                                                    uint32_t* __restrict__ start)
{
    __shared__ uint32_t sums[1024];
    const int per = (nbins + 1023) / 1024;
    const int tid = (int)threadIdx.x;
    const int lo = min(tid * per, nbins), hi = min(lo + per, nbins);
    uint32_t s = 0;
    for (int i = lo; i < hi; ++i) s += totals[i];
    sums[threadIdx.x] = s;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        const uint32_t v = threadIdx.x >= (unsigned)off ? sums[threadIdx.x - off] : 0u;
        __syncthreads();
        sums[threadIdx.x] += v;
        __syncthreads();
    }
    uint32_t run = threadIdx.x ? sums[threadIdx.x - 1] : 0u;
    for (int i = lo; i < hi; ++i) {
        start[i] = run;
        run += totals[i];
    }
    if (threadIdx.x == 1023) start[nbins] = sums[1023];
}

// In place: hist[b][bin] <- start[bin] + sum_{b' < b} hist[b'][bin].
__global__ __launch_bounds__(256) void offsets_kernel(uint32_t* __restrict__ hist, int nblocks,
                                                      int nbins, int nchunks,
                                                      const uint32_t* __restrict__ csum,
                                                      const uint32_t* __restrict__ start)
{
    const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= (int64_t)nbins * nchunks) return;
    const int c = (int)(id / nbins), bin = (int)(id - (int64_t)c * nbins);
    const int b0 = c * kScanChunk, b1 = min(b0 + kScanChunk, nblocks);
    uint32_t run = start[bin] + csum[(size_t)c * nbins + bin];
    for (int b = b0; b < b1; ++b) {
        const uint32_t v = hist[(size_t)b * nbins + bin];
        hist[(size_t)b * nbins + bin] = run;
        run += v;
    }
}

template <int RM>
__global__ __launch_bounds__(kBinThreads) void fwd_scatter_kernel(
    WinParams P, TileGeom G, const float* __restrict__ ex, const float* __restrict__ ey,
    const float* __restrict__ et, const int8_t* __restrict__ ep, int64_t n,
    const float* __restrict__ rho, const float* __restrict__ ego,
    const uint32_t* __restrict__ offs, SplatRec* __restrict__ rec)
{
    const FlowSrc u = flow_src(P, rho, ego);
    extern __shared__ uint32_t lh[];
    const uint32_t* row = offs + (size_t)blockIdx.x * G.nbins;
    for (int i = threadIdx.x; i < G.nbins; i += blockDim.x) lh[i] = row[i];
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * kBinThreads * G.ept;
    for (int e = 0; e < G.ept; ++e) {
        const int64_t k = base + (int64_t)e * kBinThreads + threadIdx.x;
        if (k >= n) break;
        double px[RM], py[RM];
        int mb;
        const float tk = et[k];
        if (!warp_event<RM>(P, u, ex[k], ey[k], tk, px, py, mb)) continue;
        const float ts = ep[k] > 0 ? tk : -tk;      // t >= 0 here; sign bit = negative polarity
        for_each_splat<RM>(P, G, px, py, [&](int bin, int r) {
            const uint32_t slot = atomicAdd(&lh[bin], 1u);
            SplatRec q;
            q.X = sel(px, r);
            q.Y = sel(py, r);
            q.ts = ts;
            q.k = (uint32_t)k;
            rec[slot] = q;
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

__device__ __forceinline__ void bin_tile(const TileGeom& G, int bin, int& r, int& tx, int& ty)
{
    r = bin / G.ntiles;
    const int tile = bin - r * G.ntiles;
    ty = tile / G.ntx;
    tx = tile - ty * G.ntx;
}

__global__ __launch_bounds__(256) void fwd_tile_kernel(WinParams P, TileGeom G,
                                                       const SplatRec* __restrict__ rec,
                                                       const uint32_t* __restrict__ start,
                                                       double2* __restrict__ img,
                                                       double2* __restrict__ halo,
                                                       double* __restrict__ part)
{
    __shared__ double2 lds[2 * TLW * TLH];
    __shared__ double red[16];
    const int bin = blockIdx.x;
    int r, tx, ty;
    bin_tile(G, bin, r, tx, ty);
    const int xo = tx * TW, yo = ty * TH;
    for (int i = threadIdx.x; i < 2 * TLW * TLH; i += blockDim.x) lds[i] = make_double2(0.0, 0.0);
    __syncthreads();
    const double ref = P.refs[r];
    const uint32_t s0 = start[bin], s1 = start[bin + 1];
    for (uint32_t i = s0 + threadIdx.x; i < s1; i += blockDim.x) {
        const SplatRec q = rec[i];
        const int pol = (__float_as_uint(q.ts) >> 31) ? 1 : 0;
        const double tb = 1.0 - fabs(ref - (double)fabsf(q.ts));
        const Taps tp = make_taps(P, q.X, q.Y);
        const int lx = tp.x0 - xo, ly = tp.y0 - yo;
        double2* L = lds + pol * TLW * TLH;
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            if (!tap_in(tp, c)) continue;
            const double w = tap_w(tp, c);
            if (w == 0.0) continue;
            double2* cell = L + (ly + (c >> 1)) * TLW + lx + (c & 1);
            atomicAdd(&cell->x, w);
            atomicAdd(&cell->y, w * tb);
        }
    }
    __syncthreads();
    double sum = 0.0, cnt = 0.0;
    double2* plane0 = img + (size_t)(r * 2 + 0) * P.HW;
    double2* plane1 = img + (size_t)(r * 2 + 1) * P.HW;
    for (int i = threadIdx.x; i < TW * TH; i += blockDim.x) {
        const int lx = i % TW, ly = i / TW;
        const int X = xo + lx, Y = yo + ly;
        if (X >= P.W || Y >= P.H) continue;
        const double2 a = lds[ly * TLW + lx], b = lds[TLW * TLH + ly * TLW + lx];
        const int pix = Y * P.W + X;
        plane0[pix] = a;
        plane1[pix] = b;
        if (lx > 0 && ly > 0) reduce_pixel(a, b, P.eps, sum, cnt);
    }
    double2* hb = halo + (size_t)bin * NHALO * 2;
    for (int j = threadIdx.x; j < NHALO; j += blockDim.x) {
        const int idx = (j <= TH) ? j * TLW + TW : TH * TLW + (j - (TH + 1));
        hb[j * 2 + 0] = lds[idx];
        hb[j * 2 + 1] = lds[TLW * TLH + idx];
    }
    sum = block_sum(sum, red);
    cnt = block_sum(cnt, red);
    if (threadIdx.x == 0) {
        part[((size_t)bin * 2 + 0) * 2 + 0] = sum;
        part[((size_t)bin * 2 + 0) * 2 + 1] = cnt;
    }
}

// Column 0 and row 0 of each tile: add the halos of the left, top and
// top-left tiles (in that order), store, and reduce those pixels.
__global__ __launch_bounds__(64) void fwd_merge_kernel(WinParams P, TileGeom G,
                                                       double2* __restrict__ img,
                                                       const double2* __restrict__ halo,
                                                       double* __restrict__ part)
{
    __shared__ double red[16];
    const int bin = blockIdx.x;
    int r, tx, ty;
    bin_tile(G, bin, r, tx, ty);
    const int xo = tx * TW, yo = ty * TH;
    double sum = 0.0, cnt = 0.0;
    for (int j = threadIdx.x; j < NBORDER; j += blockDim.x) {
        const int lx = j < TH ? 0 : j - TH + 1;
        const int ly = j < TH ? j : 0;
        const int X = xo + lx, Y = yo + ly;
        if (X >= P.W || Y >= P.H) continue;
        const int pix = Y * P.W + X;
        double2 v[2];
#pragma unroll
        for (int pol = 0; pol < 2; ++pol) {
            double2 a = img[(size_t)(r * 2 + pol) * P.HW + pix];
            if (lx == 0 && tx > 0) {
                const double2 h = halo[((size_t)(bin - 1) * NHALO + ly) * 2 + pol];
                a.x += h.x;
                a.y += h.y;
            }
            if (ly == 0 && ty > 0) {
                const double2 h = halo[((size_t)(bin - G.ntx) * NHALO + TH + 1 + lx) * 2 + pol];
                a.x += h.x;
                a.y += h.y;
            }
            if (lx == 0 && ly == 0 && tx > 0 && ty > 0) {
                const double2 h = halo[((size_t)(bin - G.ntx - 1) * NHALO + TH) * 2 + pol];
                a.x += h.x;
                a.y += h.y;
            }
            img[(size_t)(r * 2 + pol) * P.HW + pix] = a;
            v[pol] = a;
        }
        reduce_pixel(v[0], v[1], P.eps, sum, cnt);
    }
    sum = block_sum(sum, red);
    cnt = block_sum(cnt, red);
    if (threadIdx.x == 0) {
        part[((size_t)bin * 2 + 1) * 2 + 0] = sum;
        part[((size_t)bin * 2 + 1) * 2 + 1] = cnt;
    }
}

// ---------------------------------------------------------------------------
// Backward: one record per flow-sampling position.  The forward sweep into
// reference r samples the flow at the previous position (the event for the
// first step), the backward sweep likewise; both first steps sample at the
// event, so their contributions share one record.
// ---------------------------------------------------------------------------

struct SweepShape {
    int rs;   // first reference of the forward sweep (skips a reference equal to t_k)
    int mb;   // references before t_k (the backward sweep visits mb-1 .. 0)
};

__device__ __forceinline__ SweepShape sweep_shape(const WinParams& P, int mb, double tk)
{
    SweepShape s;
    s.mb = mb;
    s.rs = (mb < P.R && P.refs[mb] == tk) ? mb + 1 : mb;
    return s;
}

// fn(X, Y) for every sampling position that is a reference position, then
// fn(x0, y0) once for the event if it takes any step.
template <int RM, typename F>
__device__ __forceinline__ void for_each_sample(const WinParams& P, const SweepShape& s,
                                                const double (&px)[RM], const double (&py)[RM],
                                                double x0, double y0, F&& fn)
{
    for (int r = s.rs + 1; r < P.R; ++r) fn(sel(px, r - 1), sel(py, r - 1));
    for (int r = s.mb - 2; r >= 0; --r) fn(sel(px, r + 1), sel(py, r + 1));
    if (s.rs < P.R || s.mb > 0) fn(x0, y0);
}

template <int RM>
__global__ __launch_bounds__(kBinThreads) void bwd_count_kernel(
    WinParams P, TileGeom G, const float* __restrict__ ex, const float* __restrict__ ey,
    const float* __restrict__ et, int64_t n, const float* __restrict__ rho,
    const float* __restrict__ ego, uint32_t* __restrict__ hist)
{
    const FlowSrc u = flow_src(P, rho, ego);
    extern __shared__ uint32_t lh[];
    for (int i = threadIdx.x; i < G.nbins; i += blockDim.x) lh[i] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * kBinThreads * G.ept;
    for (int e = 0; e < G.ept; ++e) {
        const int64_t k = base + (int64_t)e * kBinThreads + threadIdx.x;
        if (k >= n) break;
        double px[RM], py[RM];
        int mb;
        const double x0 = ex[k], y0 = ey[k], tk = et[k];
        if (!warp_event<RM>(P, u, x0, y0, tk, px, py, mb)) continue;
        const SweepShape s = sweep_shape(P, mb, tk);
        for_each_sample<RM>(P, s, px, py, x0, y0, [&](double X, double Y) {
            atomicAdd(&lh[tile_index(G, make_taps(P, X, Y))], 1u);
        });
    }
    __syncthreads();
    uint32_t* row = hist + (size_t)blockIdx.x * G.nbins;
    for (int i = threadIdx.x; i < G.nbins; i += blockDim.x) row[i] = lh[i];
}

template <int RM>
__global__ __launch_bounds__(kBinThreads) void bwd_sweep_kernel(
    WinParams P, TileGeom G, const float* __restrict__ ex, const float* __restrict__ ey,
    const float* __restrict__ et, const int8_t* __restrict__ ep, int64_t n,
    const float* __restrict__ rho, const float* __restrict__ ego,
    const double* __restrict__ img, const StateHeader* __restrict__ hdr,
    const uint32_t* __restrict__ offs, GradRec* __restrict__ rec)
{
    const FlowSrc u = flow_src(P, rho, ego);
    extern __shared__ uint32_t lh[];
    const uint32_t* row = offs + (size_t)blockIdx.x * G.nbins;
    for (int i = threadIdx.x; i < G.nbins; i += blockDim.x) lh[i] = row[i];
    __syncthreads();
    double coef[RM];
#pragma unroll
    for (int r = 0; r < RM; ++r) coef[r] = r < P.R ? P.two_over_R / (hdr->nact[r] + P.eps) : 0.0;
    const int64_t base = (int64_t)blockIdx.x * kBinThreads * G.ept;

    auto emit = [&](double X, double Y, double gx, double gy) {
        const uint32_t slot = atomicAdd(&lh[tile_index(G, make_taps(P, X, Y))], 1u);
        GradRec q;
        q.X = X;
        q.Y = Y;
        q.gx = gx;
        q.gy = gy;
        rec[slot] = q;
    };

    for (int e = 0; e < G.ept; ++e) {
        const int64_t k = base + (int64_t)e * kBinThreads + threadIdx.x;
        if (k >= n) break;
        double px[RM], py[RM];
        int mb;
        const double x0 = ex[k], y0 = ey[k], tk = et[k];
        if (!warp_event<RM>(P, u, x0, y0, tk, px, py, mb)) continue;
        const int pol = ep[k] > 0 ? 0 : 1;
        const double2* planes = reinterpret_cast<const double2*>(img) + (size_t)pol * P.HW;
        const SweepShape sh = sweep_shape(P, mb, tk);
        const int nv = (P.R - sh.rs) + mb;
        double g0x = 0.0, g0y = 0.0;     // contributions sampled at the event position
        double Lx = 0.0, Ly = 0.0;
        for (int j = 0; j < nv; ++j) {
            const ReverseStep s = reverse_step<RM>(P, j, sh.rs, mb, x0, y0, tk, px, py);
            if (s.restart) {
                Lx = 0.0;
                Ly = 0.0;
            }
            direct_term(P, planes + (size_t)s.r * 2 * P.HW, sel(coef, s.r),
                        1.0 - fabs(P.refs[s.r] - tk), sel(px, s.r), sel(py, s.r), Lx, Ly);
            if (s.first) {
                g0x += s.dt * Lx;
                g0y += s.dt * Ly;
            } else {
                emit(s.X, s.Y, s.dt * Lx, s.dt * Ly);
                double jx, jy;
                jacobian_t(P, u, s.X, s.Y, Lx, Ly, jx, jy);
                Lx += s.dt * jx;
                Ly += s.dt * jy;
            }
        }
        if (nv > 0) emit(x0, y0, g0x, g0y);
    }
}

// Accumulate dL/du = sum over records of w_tap * (dt * adjoint) in LDS; own
// pixels off the border get d rho and their d theta share here, the border
// and the halo go to buffers for the merge.
__global__ __launch_bounds__(256) void bwd_tile_kernel(
    WinParams P, TileGeom G, const GradRec* __restrict__ rec, const uint32_t* __restrict__ start,
    const float* __restrict__ rho, const float* __restrict__ ego,
    const float* __restrict__ grad_loss, float* __restrict__ drho,
    double2* __restrict__ halo, double2* __restrict__ border, double* __restrict__ part)
{
    __shared__ double2 lds[TLW * TLH];
    __shared__ double red[16];
    const int tile = blockIdx.x;
    const int ty = tile / G.ntx, tx = tile - ty * G.ntx;
    const int xo = tx * TW, yo = ty * TH;
    for (int i = threadIdx.x; i < TLW * TLH; i += blockDim.x) lds[i] = make_double2(0.0, 0.0);
    __syncthreads();
    const uint32_t s0 = start[tile], s1 = start[tile + 1];
    for (uint32_t i = s0 + threadIdx.x; i < s1; i += blockDim.x) {
        const GradRec q = rec[i];
        const Taps tp = make_taps(P, q.X, q.Y);
        const int lx = tp.x0 - xo, ly = tp.y0 - yo;
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            if (!tap_in(tp, c)) continue;
            const double w = tap_w(tp, c);
            if (w == 0.0) continue;
            double2* cell = lds + (ly + (c >> 1)) * TLW + lx + (c & 1);
            atomicAdd(&cell->x, w * q.gx);
            atomicAdd(&cell->y, w * q.gy);
        }
    }
    __syncthreads();
    const Motion m = load_motion(P, ego);
    const double gl = (double)grad_loss[0];
    double dth[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    for (int i = threadIdx.x; i < TW * TH; i += blockDim.x) {
        const int lx = i % TW, ly = i / TW;
        const int X = xo + lx, Y = yo + ly;
        if (X >= P.W || Y >= P.H) continue;
        const double2 g = lds[ly * TLW + lx];
        if (lx == 0 || ly == 0) {
            border[(size_t)tile * NBORDER + (lx == 0 ? ly : TH + lx - 1)] = g;
            continue;
        }
        const int pix = Y * P.W + X;
        double Ax, Ay, Bx, By;
        flow_parts(P, m, X, Y, Ax, Ay, Bx, By);
        drho[pix] = (float)(gl * (g.x * Bx + g.y * By));
        if (g.x != 0.0 || g.y != 0.0) dtheta_at_pixel(P, X, Y, (double)rho[pix], g.x, g.y, dth);
    }
    double2* hb = halo + (size_t)tile * NHALO;
    for (int j = threadIdx.x; j < NHALO; j += blockDim.x) {
        const int idx = (j <= TH) ? j * TLW + TW : TH * TLW + (j - (TH + 1));
        hb[j] = lds[idx];
    }
#pragma unroll
    for (int c = 0; c < 6; ++c) {
        const double v = block_sum(dth[c], red);
        if (threadIdx.x == 0) part[(size_t)tile * 12 + c] = v;
    }
}

__global__ __launch_bounds__(64) void bwd_merge_kernel(
    WinParams P, TileGeom G, const float* __restrict__ rho, const float* __restrict__ ego,
    const float* __restrict__ grad_loss, float* __restrict__ drho,
    const double2* __restrict__ halo, const double2* __restrict__ border,
    double* __restrict__ part)
{
    __shared__ double red[16];
    const int tile = blockIdx.x;
    const int ty = tile / G.ntx, tx = tile - ty * G.ntx;
    const int xo = tx * TW, yo = ty * TH;
    const Motion m = load_motion(P, ego);
    const double gl = (double)grad_loss[0];
    double dth[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    for (int j = threadIdx.x; j < NBORDER; j += blockDim.x) {
        const int lx = j < TH ? 0 : j - TH + 1;
        const int ly = j < TH ? j : 0;
        const int X = xo + lx, Y = yo + ly;
        if (X >= P.W || Y >= P.H) continue;
        double2 g = border[(size_t)tile * NBORDER + j];
        if (lx == 0 && tx > 0) {
            const double2 h = halo[(size_t)(tile - 1) * NHALO + ly];
            g.x += h.x;
            g.y += h.y;
        }
        if (ly == 0 && ty > 0) {
            const double2 h = halo[(size_t)(tile - G.ntx) * NHALO + TH + 1 + lx];
            g.x += h.x;
            g.y += h.y;
        }
        if (lx == 0 && ly == 0 && tx > 0 && ty > 0) {
            const double2 h = halo[(size_t)(tile - G.ntx - 1) * NHALO + TH];
            g.x += h.x;
            g.y += h.y;
        }
        const int pix = Y * P.W + X;
        double Ax, Ay, Bx, By;
        flow_parts(P, m, X, Y, Ax, Ay, Bx, By);
        drho[pix] = (float)(gl * (g.x * Bx + g.y * By));
        if (g.x != 0.0 || g.y != 0.0) dtheta_at_pixel(P, X, Y, (double)rho[pix], g.x, g.y, dth);
    }
#pragma unroll
    for (int c = 0; c < 6; ++c) {
        const double v = block_sum(dth[c], red);
        if (threadIdx.x == 0) part[(size_t)tile * 12 + 6 + c] = v;
    }
}

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------

TileGeom tile_geom(const WinParams& P, int64_t n, bool forward)
{
    TileGeom G;
    G.ntx = (P.W + TW - 1) / TW;
    G.nty = (P.H + TH - 1) / TH;
    G.ntiles = G.ntx * G.nty;
    G.nbins = forward ? P.R * G.ntiles : G.ntiles;
    // enough blocks to fill the chip, few enough to keep the histogram matrix small
    int64_t ept = n / ((int64_t)kBinThreads * 1024);
    G.ept = (int)std::max<int64_t>(1, std::min<int64_t>(ept, kMaxEventsPerThread));
    const int64_t per_block = (int64_t)kBinThreads * G.ept;
    G.nblocks = (int)std::max<int64_t>(1, (n + per_block - 1) / per_block);
    return G;
}

bool tiled_supported(const WinParams& P, int64_t n)
{
    const TileGeom G = tile_geom(P, n, true);
    return G.nbins <= kMaxBins && n * (int64_t)P.R < (int64_t)1 << 31;
}

TileWorkspace tile_workspace_layout(const WinParams& P, int64_t n)
{
    const TileGeom G = tile_geom(P, n, true);
    TileWorkspace W;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off += (bytes + 255) / 256 * 256;
        return o;
    };
    W.hist = take((size_t)G.nblocks * G.nbins * sizeof(uint32_t));
    W.csum = take((size_t)((G.nblocks + kScanChunk - 1) / kScanChunk) * G.nbins * sizeof(uint32_t));
    W.totals = take((size_t)(G.nbins + 1) * sizeof(uint32_t));
    W.start = take((size_t)(G.nbins + 1) * sizeof(uint32_t));
    W.part = take((size_t)std::max(G.nbins * 4, G.ntiles * 12) * sizeof(double));
    W.halo = take((size_t)std::max<size_t>((size_t)G.nbins * NHALO * 2,
                                           (size_t)G.ntiles * (NHALO + NBORDER)) *
                  sizeof(double2));
    W.records = take((size_t)n * P.R * std::max(sizeof(SplatRec), sizeof(GradRec)));
    W.total = off;
    return W;
}

static hipError_t sort_bins(const TileGeom& G, uint32_t* hist, uint32_t* csum, uint32_t* totals,
                            uint32_t* start, hipStream_t s, Profiler* prof, int phase)
{
    PhaseScope ph(prof, phase, s);
    const int nchunks = (G.nblocks + kScanChunk - 1) / kScanChunk;
    const int64_t cells = (int64_t)G.nbins * nchunks;
    const int gc = (int)((cells + 255) / 256);
    chunk_sum_kernel<<<gc, 256, 0, s>>>(hist, G.nblocks, G.nbins, nchunks, csum);
    chunk_scan_kernel<<<(G.nbins + 255) / 256, 256, 0, s>>>(csum, G.nbins, nchunks, totals);
    scan_kernel<<<1, 1024, 0, s>>>(totals, G.nbins, start);
    offsets_kernel<<<gc, 256, 0, s>>>(hist, G.nblocks, G.nbins, nchunks, csum, start);
    return hipGetLastError();
}

template <int RM>
static hipError_t tiled_forward_rm(const WinParams& P, const EventPtrs& ev, const float* rho,
                                   const float* ego, float* loss, const StatePtrs& st,
                                   char* ws, const TileWorkspace& W, hipStream_t s,
                                   Profiler* prof)
{
    const TileGeom G = tile_geom(P, ev.n, true);
    uint32_t* hist = reinterpret_cast<uint32_t*>(ws + W.hist);
    uint32_t* totals = reinterpret_cast<uint32_t*>(ws + W.totals);
    uint32_t* csum = reinterpret_cast<uint32_t*>(ws + W.csum);
    uint32_t* start = reinterpret_cast<uint32_t*>(ws + W.start);
    double* part = reinterpret_cast<double*>(ws + W.part);
    double2* halo = reinterpret_cast<double2*>(ws + W.halo);
    SplatRec* rec = reinterpret_cast<SplatRec*>(ws + W.records);
    double2* img = reinterpret_cast<double2*>(st.img);
    const size_t lds = (size_t)G.nbins * sizeof(uint32_t);
    hipError_t e;
    {
        PhaseScope ph(prof, kPhZero, s);   // only the per-window sums need clearing
        e = launch_fill_zero(reinterpret_cast<float*>(st.hdr), sizeof(StateHeader) / 4, s);
    }
    if (e != hipSuccess) return e;
    {
        PhaseScope ph(prof, kPhCount, s);
        fwd_count_kernel<RM><<<G.nblocks, kBinThreads, lds, s>>>(P, G, ev.x, ev.y, ev.t, ev.n,
                                                                 rho, ego, hist, &st.hdr->n_valid);
        e = hipGetLastError();
    }
    if (e != hipSuccess) return e;
    if ((e = sort_bins(G, hist, csum, totals, start, s, prof, kPhScan)) != hipSuccess) return e;
    {
        PhaseScope ph(prof, kPhScatter, s);
        fwd_scatter_kernel<RM><<<G.nblocks, kBinThreads, lds, s>>>(P, G, ev.x, ev.y, ev.t, ev.p,
                                                                   ev.n, rho, ego, hist, rec);
        e = hipGetLastError();
    }
    if (e != hipSuccess) return e;
    {
        PhaseScope ph(prof, kPhSplat, s);
        fwd_tile_kernel<<<G.nbins, 256, 0, s>>>(P, G, rec, start, img, halo, part);
        e = hipGetLastError();
    }
    if (e != hipSuccess) return e;
    {
        PhaseScope ph(prof, kPhReduce, s);
        fwd_merge_kernel<<<G.nbins, 64, 0, s>>>(P, G, img, halo, part);
        e = hipGetLastError();
    }
    if (e != hipSuccess) return e;
    {
        PhaseScope ph(prof, kPhFinalize, s);
        finalize_forward_kernel<<<1, 256, 0, s>>>(P, part, 2 * G.ntiles, st.hdr, loss);
        e = hipGetLastError();
    }
    return e;
}

hipError_t launch_forward_tiled(const WinParams& P, const EventPtrs& ev, const float* rho,
                                const float* ego, float* loss, const StatePtrs& st, char* ws,
                                hipStream_t s, Profiler* prof)
{
    const TileWorkspace W = tile_workspace_layout(P, ev.n);
    if (P.R <= 2) return tiled_forward_rm<2>(P, ev, rho, ego, loss, st, ws, W, s, prof);
    if (P.R <= 4) return tiled_forward_rm<4>(P, ev, rho, ego, loss, st, ws, W, s, prof);
    if (P.R <= 8) return tiled_forward_rm<8>(P, ev, rho, ego, loss, st, ws, W, s, prof);
    return tiled_forward_rm<16>(P, ev, rho, ego, loss, st, ws, W, s, prof);
}

template <int RM>
static hipError_t tiled_backward_rm(const WinParams& P, const EventPtrs& ev, const float* rho,
                                    const float* ego, const StatePtrs& st, const float* grad_loss,
                                    float* grad_rho, float* grad_ego, char* ws,
                                    const TileWorkspace& W, hipStream_t s, Profiler* prof)
{
    const TileGeom G = tile_geom(P, ev.n, false);
    uint32_t* hist = reinterpret_cast<uint32_t*>(ws + W.hist);
    uint32_t* totals = reinterpret_cast<uint32_t*>(ws + W.totals);
    uint32_t* csum = reinterpret_cast<uint32_t*>(ws + W.csum);
    uint32_t* start = reinterpret_cast<uint32_t*>(ws + W.start);
    double* part = reinterpret_cast<double*>(ws + W.part);
    double2* halo = reinterpret_cast<double2*>(ws + W.halo);
    double2* border = halo + (size_t)G.ntiles * NHALO;
    GradRec* rec = reinterpret_cast<GradRec*>(ws + W.records);
    const size_t lds = (size_t)G.nbins * sizeof(uint32_t);
    hipError_t e;
    {
        PhaseScope ph(prof, kPhGradCount, s);
        bwd_count_kernel<RM><<<G.nblocks, kBinThreads, lds, s>>>(P, G, ev.x, ev.y, ev.t, ev.n,
                                                                 rho, ego, hist);
        e = hipGetLastError();
    }
    if (e != hipSuccess) return e;
    if ((e = sort_bins(G, hist, csum, totals, start, s, prof, kPhGradScan)) != hipSuccess) return e;
    {
        PhaseScope ph(prof, kPhAdjoint, s);
        bwd_sweep_kernel<RM><<<G.nblocks, kBinThreads, lds, s>>>(
            P, G, ev.x, ev.y, ev.t, ev.p, ev.n, rho, ego, st.img, st.hdr, hist, rec);
        e = hipGetLastError();
    }
    if (e != hipSuccess) return e;
    {
        PhaseScope ph(prof, kPhGradTile, s);
        bwd_tile_kernel<<<G.ntiles, 256, 0, s>>>(P, G, rec, start, rho, ego, grad_loss, grad_rho,
                                                 halo, border, part);
        bwd_merge_kernel<<<G.ntiles, 64, 0, s>>>(P, G, rho, ego, grad_loss, grad_rho, halo,
                                                 border, part);
        e = hipGetLastError();
    }
    if (e != hipSuccess) return e;
    {
        PhaseScope ph(prof, kPhGradFinalize, s);
        finalize_backward_kernel<<<1, 256, 0, s>>>(part, 2 * G.ntiles, grad_loss, grad_ego);
        e = hipGetLastError();
    }
    return e;
}

hipError_t launch_backward_tiled(const WinParams& P, const EventPtrs& ev, const float* rho,
                                 const float* ego, const StatePtrs& st, const float* grad_loss,
                                 float* grad_rho, float* grad_ego, char* ws, hipStream_t s,
                                 Profiler* prof)
{
    const TileWorkspace W = tile_workspace_layout(P, ev.n);
    if (P.R <= 2) return tiled_backward_rm<2>(P, ev, rho, ego, st, grad_loss, grad_rho, grad_ego, ws, W, s, prof);
    if (P.R <= 4) return tiled_backward_rm<4>(P, ev, rho, ego, st, grad_loss, grad_rho, grad_ego, ws, W, s, prof);
    if (P.R <= 8) return tiled_backward_rm<8>(P, ev, rho, ego, st, grad_loss, grad_rho, grad_ego, ws, W, s, prof);
    return tiled_backward_rm<16>(P, ev, rho, ego, st, grad_loss, grad_rho, grad_ego, ws, W, s, prof);
}

}  // namespace cm
