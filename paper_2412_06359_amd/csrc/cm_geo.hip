// cm_geo.hip -- geometry-consistency loss between consecutive flow sets
// (paper Sec. 3.2, Eq. 3) and the full loss L = L_CM + lambda L_geo (Eq. 4),
// forward and backward, for one window or a batch.
//
// Pair f of a window (flow sets f and f+1, f = 0 .. F-2): pixel x = (i, j) of
// set f, with inverse depth rho_a = rho_f(x) > 0, moves with segment f's
// motion, rotation Exp(Delta_f w_f) and translation Delta_f v_f
// (Delta_f = k_{f+1} - k_f, the segment's length):
//   x0 = ((i - cx)/fx, (j - cy)/fy, 1),   p = R x0 + rho_a t   (= rho_a P),
//   D_{0->1} = a = p_z / rho_a,           x' = i + fx (p_x/p_z - x0_x), ...
// (x' in this form maps every pixel exactly onto itself at zero motion), and
// D'_1 = b = sum over the on-sensor taps of x' of w_q / rho_{f+1}(tap).  The
// pixel is in V if p_z > 0, x' lies in the closed image box and every
// on-sensor tap has rho_{f+1} > 0.  L_geo = mean over pairs of the pair's mean
// over V of |a - b| / (a + b); one flow set gives L_geo = 0.
//
// Work per pixel and pair: a coalesced read of rho_a, a 4-tap gather of
// rho_{f+1} near x', the rotation and projection of one ray in FP64 (the FP64
// ALU, not HBM, bounds it).  A block takes a 32 x 32 tile of one (window,
// pair); grid (tiles, windows, pairs).
//
// Reductions run in a fixed order (per thread in pixel order, 64-lane tree,
// waves in order, tiles in order), so the forward is deterministic.  In the
// backward, a pixel's own d rho_a has one writer; the d rho_{f+1} at its taps
// is a scatter.  A block gathers its tile's scatter in a 64 x 64 LDS window
// centred on the projection of the tile's centre and adds each touched cell
// to memory once (taps outside the window go to memory directly).  The
// deterministic mode accumulates the scatter in 64-bit fixed point (integer
// addition is associative), with a per-pair scale chosen from a bound the
// forward records, and adds it to d rho in a separate pass; the atomic mode
// accumulates in FP64 in LDS and adds floats to memory.
#include "cm_kernels.hpp"

namespace cm {

namespace {

constexpr int kGeoThreads = 256;
constexpr int kGeoTile = 32;                          // tile side (pixels)
constexpr int kGeoRows = kGeoThreads / kGeoTile;      // tile rows per pass
constexpr int kGeoPasses = kGeoTile / kGeoRows;       // pixels per thread
constexpr int kGeoWin = 64;                           // LDS scatter window side
constexpr int kApplyPix = 1024;                       // pixels per apply block

// Knot k of a window: {0, 1} U refs in increasing order.
__device__ __forceinline__ double knot_of(const WinParams& P, int k)
{
    const int k0 = P.refs[0] > 0.0 ? 1 : 0;
    if (k < k0) return 0.0;
    if (k - k0 < P.R) return P.refs[k - k0];
    return 1.0;
}

struct GeoPose {
    double R[9];
    double Jr[9];
    double t[3];
    double delta;
};

__device__ __forceinline__ GeoPose pair_pose(const WinParams& P, const float* __restrict__ ego,
                                             int f)
{
    GeoPose g;
    g.delta = knot_of(P, f + 1) - knot_of(P, f);
    rotation_exp(g.delta * (double)ego[3], g.delta * (double)ego[4], g.delta * (double)ego[5],
                 g.R, g.Jr);
    for (int k = 0; k < 3; ++k) g.t[k] = g.delta * (double)ego[k];
    return g;
}

struct GeoPix {
    double x0x, x0y;        // ray of the pixel
    double p[3];            // rho_a times the moved point
    double iz;              // 1 / p_z
    double inv_ra;          // 1 / rho_a
    Taps tp;                // taps of x'
    double ib[4];           // 1 / rho_{f+1} at the taps (0 off the sensor)
    double a, b;            // D_{0->1}, D'_1
    double inv_s;           // 1 / (a + b)
};

// Reciprocals of five positive values with one division: with
// m = x0 x1, n = x2 x3 and q = m (n x4), u = (1/q)(n x4) = 1/(x0 x1) and
// v = (1/q) m = 1/(x2 x3 x4) give 1/x0 = u x1, 1/x1 = u x0, 1/x2 = v (x3 x4),
// 1/x3 = v (x2 x4), 1/x4 = v n.  The formula is symmetric in x0 and x1, so
// equal values there get bit-equal reciprocals (x0 is the pixel's own inverse
// depth, x1 its first tap: zero motion then gives exactly D_{0->1} = D'_1).
// Where q leaves the normal range each value is divided on its own.
__device__ __forceinline__ void reciprocals5(const double (&x)[5], double (&r)[5])
{
    const double m = x[0] * x[1], n = x[2] * x[3];
    const double t = n * x[4];
    const double q = m * t;
    if (q >= 1e-290 && q <= 1e290) {
        const double inv = 1.0 / q;
        const double u = inv * t, v = inv * m;
        r[0] = u * x[1];
        r[1] = u * x[0];
        r[2] = v * (x[3] * x[4]);
        r[3] = v * (x[2] * x[4]);
        r[4] = v * n;
    } else {
#pragma unroll
        for (int k = 0; k < 5; ++k) r[k] = 1.0 / x[k];
    }
}

__device__ __forceinline__ bool geo_pixel(const WinParams& P, const GeoPose& g, int i, int j,
                                          float ra, const float* __restrict__ rb, GeoPix& o)
{
    if (!(ra > 0.f)) return false;
    const double rho_a = (double)ra;
    o.x0x = ((double)i - P.cx) * P.inv_fx;
    o.x0y = ((double)j - P.cy) * P.inv_fy;
#pragma unroll
    for (int k = 0; k < 3; ++k)
        o.p[k] = ((g.R[3 * k] * o.x0x + g.R[3 * k + 1] * o.x0y) + g.R[3 * k + 2]) + rho_a * g.t[k];
    if (!(o.p[2] > 0.0)) return false;
    o.iz = 1.0 / o.p[2];
    const double xs = (double)i + P.fx * (o.p[0] * o.iz - o.x0x);
    const double ys = (double)j + P.fy * (o.p[1] * o.iz - o.x0y);
    if (!(xs >= 0.0 && xs <= P.xmax && ys >= 0.0 && ys <= P.ymax)) return false;
    o.tp = make_taps(P, xs, ys);
    const float* row0 = rb + (size_t)o.tp.y0 * P.W + o.tp.x0;
    int off[4];
    tap_offsets(P, o.tp, off);
    float rq[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) rq[q] = row0[off[q]];
#pragma unroll
    for (int q = 1; q < 4; ++q)
        if (!tap_in(o.tp, q)) rq[q] = 1.f;
#pragma unroll
    for (int q = 0; q < 4; ++q)
        if (!(rq[q] > 0.f)) return false;        // off-sensor taps read 1
    const double xv[5] = {rho_a, (double)rq[0], (double)rq[1], (double)rq[2], (double)rq[3]};
    double rv[5];
    reciprocals5(xv, rv);
    o.inv_ra = rv[0];
    o.b = 0.0;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        o.ib[q] = tap_in(o.tp, q) ? rv[q + 1] : 0.0;
        o.b += tap_w(o.tp, q) * o.ib[q];
    }
    o.a = o.p[2] * o.inv_ra;
    o.inv_s = 1.0 / (o.a + o.b);
    return true;
}

// Block-wide sums of N doubles per thread in one pass: 64-lane trees, then
// the waves in order (thread 0 gets the results).
template <int N>
__device__ __forceinline__ void block_sums(double (&v)[N], double* lds /* >= 4 N */)
{
#pragma unroll
    for (int c = 0; c < N; ++c)
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) v[c] += __shfl_down(v[c], o, 64);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0)
#pragma unroll
        for (int c = 0; c < N; ++c) lds[wid * N + c] = v[c];
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int c = 0; c < N; ++c) {
            double t = 0.0;
            for (int wv = 0; wv < (int)(blockDim.x >> 6); ++wv) t += lds[wv * N + c];
            v[c] = t;
        }
    }
}

// Tiles of a window.
__device__ __forceinline__ int geo_ntx(const WinParams& P) { return (P.W + kGeoTile - 1) / kGeoTile; }
__device__ __forceinline__ int geo_ntiles(const WinParams& P)
{
    return geo_ntx(P) * ((P.H + kGeoTile - 1) / kGeoTile);
}

__device__ __forceinline__ double block_max(double v, double* lds /* >= 16 */)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_down(v, o, 64));
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) lds[wid] = v;
    __syncthreads();
    double m = 0.0;
    if (threadIdx.x == 0)
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) m = fmax(m, lds[w]);
    return m;   // valid in thread 0
}

// One thread per (window, pair): the pair's pose, read by every block of it.
__global__ __launch_bounds__(64) void geo_pose_prep_kernel(const WinMeta* __restrict__ meta,
                                                           int nw, int npm,
                                                           const float* __restrict__ ego,
                                                           GeoPose* __restrict__ poses)
{
    const int id = blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= nw * npm) return;
    const int w = id / npm, f = id - w * npm;
    const WinParams& P = meta[w].P;
    if (f >= P.F - 1) return;
    poses[id] = pair_pose(P, ego + 6 * (meta[w].ego_off + f), f);
}

// Forward: per block of pixels, the sum of the terms over V, |V| and the
// bound of the fixed-point scatter, B = max |d term/db| max_q rho_{f+1}^-2.
__global__ __launch_bounds__(kGeoThreads) void geo_forward_kernel(
    const WinMeta* __restrict__ meta, int nblk, int npm, const float* __restrict__ rho,
    const GeoPose* __restrict__ poses, double* __restrict__ part)
{
    __shared__ double red[16];
    const int w = blockIdx.y, f = blockIdx.z, blk = blockIdx.x;
    const WinParams& P = meta[w].P;
    if (f >= P.F - 1 || blk >= geo_ntiles(P)) return;
    const GeoPose& g = poses[(size_t)w * npm + f];
    const float* ra = rho + meta[w].pix_off + (size_t)f * P.HW;
    const float* rb = ra + P.HW;
    const int ntx = geo_ntx(P), ty = blk / ntx, tx = blk - ty * ntx;
    const int i = tx * kGeoTile + (int)(threadIdx.x % kGeoTile);
    const int jt = ty * kGeoTile + (int)(threadIdx.x / kGeoTile);
    double sum = 0.0, cnt = 0.0, bound = 0.0;
    for (int k = 0; k < kGeoPasses; ++k) {
        const int j = jt + k * kGeoRows;
        if (i >= P.W || j >= P.H) continue;
        const int pix = j * P.W + i;
        GeoPix o;
        if (!geo_pixel(P, g, i, j, ra[pix], rb, o)) continue;
        sum += fabs(o.a - o.b) * o.inv_s;
        cnt += 1.0;
        double im = 0.0;
#pragma unroll
        for (int q = 0; q < 4; ++q) im = fmax(im, o.ib[q]);
        bound = fmax(bound, ((2.0 * o.a) * (o.inv_s * o.inv_s)) * (im * im));
    }
    double sc[2] = {sum, cnt};
    block_sums<2>(sc, red);
    sum = sc[0];
    cnt = sc[1];
    bound = block_max(bound, red + 8);
    if (threadIdx.x == 0) {
        double* q = part + (((size_t)w * npm + f) * nblk + blk) * 3;
        q[0] = sum;
        q[1] = cnt;
        q[2] = bound;
    }
}

// Per window: pair means, |V|, fixed-point scales; L_geo and Eq. 4.  Wave v
// reduces pairs v, v + 4, ... (fixed order), thread 0 sums the pair means.
__global__ __launch_bounds__(256) void geo_finalize_kernel(
    const WinMeta* __restrict__ meta, int nblk, int npm, const double* __restrict__ part,
    GeoPairSum* __restrict__ pairs, float lambda, const float* __restrict__ loss_cm,
    float* __restrict__ loss_geo, float* __restrict__ loss_total)
{
    __shared__ double means[kMaxFlows];
    const int w = blockIdx.x;
    const WinParams& P = meta[w].P;
    const int nb = geo_ntiles(P);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    for (int f = wid; f < P.F - 1; f += (int)(blockDim.x >> 6)) {
        const double* q = part + ((size_t)w * npm + f) * nblk * 3;
        double s = 0.0, c = 0.0, m = 0.0;
        for (int b = lane; b < nb; b += 64) {
            s += q[3 * b];
            c += q[3 * b + 1];
            m = fmax(m, q[3 * b + 2]);
        }
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            s += __shfl_down(s, o, 64);
            c += __shfl_down(c, o, 64);
            m = fmax(m, __shfl_down(m, o, 64));
        }
        if (lane == 0) {
            GeoPairSum r;
            r.mean = c > 0.0 ? s / c : 0.0;
            r.count = c;
            // |sum of scaled contributions at a pixel| <= |V| B 2^e < 2^61
            int ex = 0;
            const double nb_bound = c * m;
            if (nb_bound > 0.0) (void)frexp(nb_bound, &ex);
            r.scale = nb_bound > 0.0 ? ldexp(1.0, 61 - ex) : 1.0;
            pairs[(size_t)w * npm + f] = r;
            means[f] = r.mean;
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double lg = 0.0;
        for (int f = 0; f < P.F - 1; ++f) lg += means[f];
        const double L = P.F > 1 ? lg / (double)(P.F - 1) : 0.0;
        loss_geo[w] = (float)L;
        if (loss_total)
            loss_total[w] = (float)((loss_cm ? (double)loss_cm[w] : 0.0) + (double)lambda * L);
    }
}

// Backward of the pairs of one parity (f = 2 blockIdx.z + parity): within a
// launch, set f is written by pair f only (its pixels' own d rho_a, a plain
// read-modify-write) and set f+1 only by pair f's scatter.  grad_rho and
// grad_ego are accumulated into (the caller's CM gradient is already there).
// DET: the scatter goes to the fixed-point buffer acc (same layout as rho);
// otherwise it is added to grad_rho as floats.
template <bool DET>
__global__ __launch_bounds__(kGeoThreads) void geo_backward_kernel(
    const WinMeta* __restrict__ meta, int nblk, int npm, int parity, const float* __restrict__ rho,
    const GeoPairSum* __restrict__ pairs, float lambda, const float* __restrict__ grad_loss,
    float* __restrict__ grad_rho, unsigned long long* __restrict__ acc,
    const GeoPose* __restrict__ poses, double* __restrict__ part)
{
    __shared__ double red[4 * 6];
    __shared__ unsigned long long win[kGeoWin * kGeoWin];   // FP64 sums or fixed point
    __shared__ int org[2];
    const int w = blockIdx.y, f = 2 * blockIdx.z + parity, blk = blockIdx.x;
    const WinParams& P = meta[w].P;
    if (f >= P.F - 1 || blk >= geo_ntiles(P)) return;
    const GeoPose& g = poses[(size_t)w * npm + f];
    const GeoPairSum pr = pairs[(size_t)w * npm + f];
    const double cf = pr.count > 0.0
                          ? (double)grad_loss[w] * (double)lambda / ((double)(P.F - 1) * pr.count)
                          : 0.0;
    const float* ra = rho + meta[w].pix_off + (size_t)f * P.HW;
    const float* rb = ra + P.HW;
    float* ga_out = grad_rho + meta[w].pix_off + (size_t)f * P.HW;
    float* gb_out = ga_out + P.HW;
    unsigned long long* acc_b = DET ? acc + meta[w].pix_off + (size_t)(f + 1) * P.HW : nullptr;
    const int ntx = geo_ntx(P), ty = blk / ntx, tx = blk - ty * ntx;
    if (threadIdx.x == 0) {
        // window origin: where the tile's centre pixel lands (the tile itself
        // where that pixel has no image)
        const int ci = min(tx * kGeoTile + kGeoTile / 2, P.W - 1);
        const int cj = min(ty * kGeoTile + kGeoTile / 2, P.H - 1);
        double xs = ci, ys = cj;
        const float rc = ra[cj * P.W + ci];
        if (rc > 0.f) {
            const double x0x = ((double)ci - P.cx) * P.inv_fx, x0y = ((double)cj - P.cy) * P.inv_fy;
            double p[3];
            for (int k = 0; k < 3; ++k)
                p[k] = ((g.R[3 * k] * x0x + g.R[3 * k + 1] * x0y) + g.R[3 * k + 2]) + (double)rc * g.t[k];
            if (p[2] > 0.0) {
                xs = (double)ci + P.fx * (p[0] / p[2] - x0x);
                ys = (double)cj + P.fy * (p[1] / p[2] - x0y);
            }
        }
        xs = fmin(fmax(xs, -65536.0), 65536.0);           // NaN-free, int-safe
        ys = fmin(fmax(ys, -65536.0), 65536.0);
        org[0] = (int)floor(xs) - (kGeoWin / 2 - 1);
        org[1] = (int)floor(ys) - (kGeoWin / 2 - 1);
    }
    for (int c = threadIdx.x; c < kGeoWin * kGeoWin; c += kGeoThreads) win[c] = 0ull;
    __syncthreads();
    const int ox = org[0], oy = org[1];
    double dp[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    if (cf != 0.0) {
        const int i = tx * kGeoTile + (int)(threadIdx.x % kGeoTile);
        const int jt = ty * kGeoTile + (int)(threadIdx.x / kGeoTile);
        for (int k = 0; k < kGeoPasses; ++k) {
            const int j = jt + k * kGeoRows;
            if (i >= P.W || j >= P.H) continue;
            const int pix = j * P.W + i;
            GeoPix o;
            const float rau = ra[pix];
            if (!geo_pixel(P, g, i, j, rau, rb, o)) continue;
            const double rho_a = (double)rau;
            const double sg = o.a > o.b ? 1.0 : (o.a < o.b ? -1.0 : 0.0);
            const double is2 = o.inv_s * o.inv_s;
            const double gbu = (-sg * 2.0 * o.a) * is2;          // d term / db
            const double ga = cf * ((sg * 2.0 * o.b) * is2);     // scaled d term / da
            const double gb = cf * gbu;
            double dbx = 0.0, dby = 0.0;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                if (!tap_in(o.tp, q)) continue;
                double dX, dY;
                tap_dw(o.tp, q, dX, dY);
                dbx += dX * o.ib[q];
                dby += dY * o.ib[q];
                const double c = gbu * tap_w(o.tp, q) * (-(o.ib[q] * o.ib[q]));
                if (c == 0.0) continue;
                const int qx = o.tp.x0 + (q & 1), qy = o.tp.y0 + (q >> 1);
                const int lx = qx - ox, ly = qy - oy;
                const bool local = (unsigned)lx < (unsigned)kGeoWin && (unsigned)ly < (unsigned)kGeoWin;
                if (DET) {
                    const unsigned long long v = (unsigned long long)(long long)llrint(c * pr.scale);
                    if (local)
                        atomicAdd(&win[ly * kGeoWin + lx], v);
                    else
                        atomicAdd(acc_b + qy * P.W + qx, v);
                } else {
                    if (local)
                        unsafeAtomicAdd(reinterpret_cast<double*>(win) + ly * kGeoWin + lx, c);
                    else
                        unsafeAtomicAdd(gb_out + qy * P.W + qx, (float)(cf * c));
                }
            }
            const double gxs = gb * dbx, gys = gb * dby;
            const double iz = o.iz;
            const double gp[3] = {gxs * P.fx * iz, gys * P.fy * iz,
                                  ga * o.inv_ra - ((gxs * P.fx * o.p[0] + gys * P.fy * o.p[1]) * iz) * iz};
            const double dra = ((gp[0] * g.t[0] + gp[1] * g.t[1]) + gp[2] * g.t[2]) -
                               (ga * o.a) * o.inv_ra;
            ga_out[pix] = (float)((double)ga_out[pix] + dra);
#pragma unroll
            for (int c = 0; c < 3; ++c) dp[c] += rho_a * gp[c];
            double sv[3];
#pragma unroll
            for (int c = 0; c < 3; ++c)
                sv[c] = (g.R[c] * gp[0] + g.R[3 + c] * gp[1]) + g.R[6 + c] * gp[2];
            const double cr[3] = {o.x0y * sv[2] - sv[1], sv[0] - o.x0x * sv[2],
                                  o.x0x * sv[1] - o.x0y * sv[0]};
#pragma unroll
            for (int c = 0; c < 3; ++c)
                dp[3 + c] += (g.Jr[c] * cr[0] + g.Jr[3 + c] * cr[1]) + g.Jr[6 + c] * cr[2];
        }
    }
    __syncthreads();
    // flush the window: one memory update per touched cell (only on-sensor
    // taps were added, the bounds check is a guard)
    for (int c = threadIdx.x; c < kGeoWin * kGeoWin; c += kGeoThreads) {
        const unsigned long long v = win[c];
        if (v == 0ull) continue;
        const int qx = ox + (c % kGeoWin), qy = oy + (c / kGeoWin);
        if ((unsigned)qx >= (unsigned)P.W || (unsigned)qy >= (unsigned)P.H) continue;
        if (DET)
            atomicAdd(acc_b + qy * P.W + qx, v);
        else
            unsafeAtomicAdd(gb_out + qy * P.W + qx, (float)(cf * __longlong_as_double((long long)v)));
    }
    block_sums<6>(dp, red);
    if (threadIdx.x == 0)
#pragma unroll
        for (int c = 0; c < 6; ++c) part[(((size_t)w * npm + f) * nblk + blk) * 6 + c] = dp[c];
}

// Deterministic mode: adds the fixed-point scatter of pair f into set f+1's
// d rho.
__global__ __launch_bounds__(kGeoThreads) void geo_apply_kernel(
    const WinMeta* __restrict__ meta, int npm, const GeoPairSum* __restrict__ pairs,
    float lambda, const float* __restrict__ grad_loss, float* __restrict__ grad_rho,
    unsigned long long* __restrict__ acc)
{
    const int w = blockIdx.y, f = blockIdx.z, blk = blockIdx.x;
    const WinParams& P = meta[w].P;
    if (f >= P.F - 1 || blk * kApplyPix >= P.HW) return;
    const GeoPairSum pr = pairs[(size_t)w * npm + f];
    const double cf = pr.count > 0.0
                          ? (double)grad_loss[w] * (double)lambda / ((double)(P.F - 1) * pr.count)
                          : 0.0;
    const double k = cf / pr.scale;
    const size_t off = meta[w].pix_off + (size_t)(f + 1) * P.HW;
    for (int e = 0; e < kApplyPix / kGeoThreads; ++e) {
        const int pix = blk * kApplyPix + e * kGeoThreads + threadIdx.x;
        if (pix >= P.HW) break;
        const long long v = (long long)acc[off + pix];
        if (v == 0) continue;
        grad_rho[off + pix] = (float)((double)grad_rho[off + pix] + (double)v * k);
    }
}

// One wavefront per (window, pair): fixed-order sum of the tiles' pose
// partials, d theta_f += Delta_f d pose.
__global__ __launch_bounds__(64) void geo_pose_kernel(const WinMeta* __restrict__ meta, int nblk,
                                                      int npm, const double* __restrict__ part,
                                                      float* __restrict__ grad_ego)
{
    const int w = blockIdx.y, f = blockIdx.x;
    const WinParams& P = meta[w].P;
    if (f >= P.F - 1) return;
    const int nb = geo_ntiles(P);
    const double* q = part + ((size_t)w * npm + f) * nblk * 6;
    double s[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    for (int b = threadIdx.x; b < nb; b += 64)
#pragma unroll
        for (int c = 0; c < 6; ++c) s[c] += q[6 * b + c];
#pragma unroll
    for (int c = 0; c < 6; ++c)
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) s[c] += __shfl_down(s[c], o, 64);
    if (threadIdx.x == 0) {
        const double delta = knot_of(P, f + 1) - knot_of(P, f);
        float* o = grad_ego + (meta[w].ego_off + f) * 6;
#pragma unroll
        for (int c = 0; c < 6; ++c) o[c] = (float)((double)o[c] + delta * s[c]);
    }
}

__global__ void fill_u64_kernel(unsigned long long* __restrict__ p, size_t n)
{
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) p[i] = 0ull;
}

}  // namespace

GeoLayout geo_layout(int nw, int max_F, int max_tiles, int max_HW, int64_t n_pixels, bool det)
{
    GeoLayout L;
    L.nblk = std::max(1, max_tiles);
    L.napply = std::max(1, (max_HW + kApplyPix - 1) / kApplyPix);
    L.npm = std::max(1, max_F - 1);
    const size_t slots = (size_t)nw * L.npm;
    size_t o = 0;
    auto take = [&](size_t bytes) {
        const size_t at = o;
        o += (bytes + 255) / 256 * 256;
        return at;
    };
    L.meta = take(sizeof(WinMeta) * (size_t)nw);
    L.part = take(sizeof(double) * slots * L.nblk * 6);
    L.pairs = take(sizeof(GeoPairSum) * slots);
    L.poses = take(sizeof(GeoPose) * slots);
    L.acc = det ? take(sizeof(unsigned long long) * (size_t)n_pixels) : 0;
    L.n_acc = det ? n_pixels : 0;
    L.det = det;
    L.total = o;
    return L;
}

hipError_t launch_geo_forward(const GeoLayout& L, const WinMeta* meta, int nw, void* state,
                              const float* rho, const float* ego, float lambda,
                              const float* loss_cm, float* loss_geo, float* loss_total,
                              hipStream_t s)
{
    char* st = static_cast<char*>(state);
    double* part = reinterpret_cast<double*>(st + L.part);
    GeoPairSum* pairs = reinterpret_cast<GeoPairSum*>(st + L.pairs);
    if (L.det)   // the backward's fixed-point accumulator starts at zero
        fill_u64_kernel<<<1024, 256, 0, s>>>(reinterpret_cast<unsigned long long*>(st + L.acc),
                                             (size_t)L.n_acc);
    GeoPose* poses = reinterpret_cast<GeoPose*>(st + L.poses);
    geo_pose_prep_kernel<<<(nw * L.npm + 63) / 64, 64, 0, s>>>(meta, nw, L.npm, ego, poses);
    geo_forward_kernel<<<dim3(L.nblk, nw, L.npm), kGeoThreads, 0, s>>>(meta, L.nblk, L.npm, rho,
                                                                       poses, part);
    geo_finalize_kernel<<<nw, 256, 0, s>>>(meta, L.nblk, L.npm, part, pairs, lambda, loss_cm,
                                           loss_geo, loss_total);
    return hipGetLastError();
}

hipError_t launch_geo_backward(const GeoLayout& L, const WinMeta* meta, int nw, void* state,
                               const float* rho, const float* ego, float lambda,
                               const float* grad_loss, float* grad_rho, float* grad_ego,
                               hipStream_t s)
{
    char* st = static_cast<char*>(state);
    double* part = reinterpret_cast<double*>(st + L.part);
    const GeoPairSum* pairs = reinterpret_cast<const GeoPairSum*>(st + L.pairs);
    unsigned long long* acc = L.det ? reinterpret_cast<unsigned long long*>(st + L.acc) : nullptr;
    GeoPose* poses = reinterpret_cast<GeoPose*>(st + L.poses);
    geo_pose_prep_kernel<<<(nw * L.npm + 63) / 64, 64, 0, s>>>(meta, nw, L.npm, ego, poses);
    const dim3 grid(L.nblk, nw, L.npm);
    for (int parity = 0; parity < 2; ++parity) {
        const int nz = (L.npm + 1 - parity) / 2;      // pairs of this parity per window
        if (nz == 0) continue;
        const dim3 gp(L.nblk, nw, nz);
        if (L.det)
            geo_backward_kernel<true><<<gp, kGeoThreads, 0, s>>>(meta, L.nblk, L.npm, parity, rho,
                                                                 pairs, lambda, grad_loss,
                                                                 grad_rho, acc, poses, part);
        else
            geo_backward_kernel<false><<<gp, kGeoThreads, 0, s>>>(meta, L.nblk, L.npm, parity,
                                                                  rho, pairs, lambda, grad_loss,
                                                                  grad_rho, nullptr, poses, part);
    }
    if (L.det)
        geo_apply_kernel<<<dim3(L.napply, nw, L.npm), kGeoThreads, 0, s>>>(meta, L.npm, pairs, lambda,
                                                                           grad_loss, grad_rho, acc);
    geo_pose_kernel<<<dim3(L.npm, nw), 64, 0, s>>>(meta, L.nblk, L.npm, part, grad_ego);
    return hipGetLastError();
}

}  // namespace cm
