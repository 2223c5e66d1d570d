// cm_device.hpp -- device-side building blocks of the CM loss kernels (gfx950).
//
// Flow from inverse depth and ego-motion (paper Eq. 2, first-order form),
// bilinear taps (the kernel kappa of Eq. 1 and the "BS" sampling of Fig. 2),
// and the per-event iterative warp of Sec. 3.1 / Sec. 3.3.
//
// All warp arithmetic is FP64: positions, flow at taps and tap weights.  The
// inputs are FP32 and widen exactly.  A position error of 1e-6 px (what FP32
// coordinates give for 100 px flows) flips whether a tiny bilinear weight is
// zero, and a weight of 1e-5 counts in Eq. 1's ratio S/(C+eps) as much as a
// weight of one; FP64 keeps those decisions on the same side as the FP64
// reference.  Image data and atomics stay FP32.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace cm {

constexpr int kMaxRefs = 16;

// Per-window constants, built on the host from the descriptor.
struct WinParams {
    int W, H, R, HW;
    double cx, cy, fx, fy;
    double inv_fx, inv_fy, fx_over_fy, fy_over_fx;
    double xmax, ymax;          // W - 1, H - 1
    double eps;
    double two_over_R;
    double refs[kMaxRefs];
};

// Ego-motion folded into the coefficients of the motion field.  With
// xb = i - cx, yb = j - cy the first-order form of Eq. 2 is
//   u = A(xb, yb) + rho * B(xb, yb)
//   A_x = fx w_y - (fx/fy) w_z yb + xb s,   A_y = -fy w_x + (fy/fx) w_z xb + yb s,
//   s   = (w_y/fx) xb - (w_x/fy) yb,
//   B_x = fx v_x - xb v_z,                  B_y = fy v_y - yb v_z.
struct Motion {
    double k0, k1, k2, k3, k4, k5;   // fx w_y, (fx/fy) w_z, w_x/fy, w_y/fx, -fy w_x, (fy/fx) w_z
    double tvx, tvy, vz;             // fx v_x, fy v_y, v_z
};

__device__ __forceinline__ Motion load_motion(const WinParams& P, const float* __restrict__ ego)
{
    const double vx = ego[0], vy = ego[1], vz = ego[2];
    const double wx = ego[3], wy = ego[4], wz = ego[5];
    Motion m;
    m.k0 = P.fx * wy;
    m.k1 = P.fx_over_fy * wz;
    m.k2 = wx * P.inv_fy;
    m.k3 = wy * P.inv_fx;
    m.k4 = -P.fy * wx;
    m.k5 = P.fy_over_fx * wz;
    m.tvx = P.fx * vx;
    m.tvy = P.fy * vy;
    m.vz = vz;
    return m;
}

// Rotational part A and translational part B of the flow at pixel (i, j).
__device__ __forceinline__ void flow_parts(const WinParams& P, const Motion& m, int i, int j,
                                           double& Ax, double& Ay, double& Bx, double& By)
{
    const double xb = (double)i - P.cx;
    const double yb = (double)j - P.cy;
    const double s = m.k3 * xb - m.k2 * yb;
    Ax = (m.k0 - m.k1 * yb) + xb * s;
    Ay = (m.k4 + m.k5 * xb) + yb * s;
    Bx = m.tvx - xb * m.vz;
    By = m.tvy - yb * m.vz;
}

__device__ __forceinline__ bool inside(const WinParams& P, double X, double Y)
{
    return X >= 0.0 && X <= P.xmax && Y >= 0.0 && Y <= P.ymax;
}

// The four bilinear taps of a position on the image.  Tap order:
// (x0,y0), (x0+1,y0), (x0,y0+1), (x0+1,y0+1).  For a position on the image
// tap 0 is always on the sensor; taps off the sensor have zero weight.
struct Taps {
    int x0, y0;
    double a, b;         // fractional parts
    bool inx, iny;       // x0+1 < W, y0+1 < H
};

__device__ __forceinline__ Taps make_taps(const WinParams& P, double X, double Y)
{
    Taps t;
    const double fx0 = floor(X), fy0 = floor(Y);
    t.x0 = (int)fx0;
    t.y0 = (int)fy0;
    t.a = X - fx0;
    t.b = Y - fy0;
    t.inx = t.x0 + 1 < P.W;
    t.iny = t.y0 + 1 < P.H;
    return t;
}

__device__ __forceinline__ bool tap_in(const Taps& t, int q)
{
    return (q & 1 ? t.inx : true) && (q & 2 ? t.iny : true);
}

__device__ __forceinline__ double tap_w(const Taps& t, int q)
{
    const double wa = (q & 1) ? t.a : 1.0 - t.a;
    const double wb = (q & 2) ? t.b : 1.0 - t.b;
    return wa * wb;
}

// d w_q / dX and d w_q / dY (floor-based formula).
__device__ __forceinline__ void tap_dw(const Taps& t, int q, double& dX, double& dY)
{
    const double wa = (q & 1) ? t.a : 1.0 - t.a;
    const double wb = (q & 2) ? t.b : 1.0 - t.b;
    dX = (q & 1) ? wb : -wb;
    dY = (q & 2) ? wa : -wa;
}

__device__ __forceinline__ int tap_pix(const WinParams& P, const Taps& t, int q)
{
    return (t.y0 + (q >> 1)) * P.W + t.x0 + (q & 1);
}

// BS(u)(X, Y): the flow sampled bilinearly at a position on the image.
__device__ __forceinline__ void sample_flow(const WinParams& P, const Motion& m,
                                            const float* __restrict__ rho, double X, double Y,
                                            double& ux, double& uy)
{
    const Taps t = make_taps(P, X, Y);
    ux = 0.0;
    uy = 0.0;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        if (!tap_in(t, q)) continue;
        const int i = t.x0 + (q & 1), j = t.y0 + (q >> 1);
        double Ax, Ay, Bx, By;
        flow_parts(P, m, i, j, Ax, Ay, Bx, By);
        const double r = (double)rho[j * P.W + i];
        const double w = tap_w(t, q);
        ux += w * (Ax + r * Bx);
        uy += w * (Ay + r * By);
    }
}

// Select / insert into small register arrays with a per-lane index (a chain of
// conditional moves, so the arrays stay in VGPRs).
template <int N>
__device__ __forceinline__ double sel(const double (&a)[N], int i)
{
    double r = a[0];
#pragma unroll
    for (int q = 1; q < N; ++q) r = (i == q) ? a[q] : r;
    return r;
}

template <int N>
__device__ __forceinline__ void put(double (&a)[N], int i, double v)
{
#pragma unroll
    for (int q = 0; q < N; ++q) a[q] = (i == q) ? v : a[q];
}

// Number of reference times strictly before t.
__device__ __forceinline__ int refs_before(const WinParams& P, double t)
{
    int m = 0;
#pragma unroll
    for (int r = 0; r < kMaxRefs; ++r) m += (r < P.R && P.refs[r] < t) ? 1 : 0;
    return m;
}

// Sec. 3.1 / 3.3: push one event through the reference times, forward for
// those after t_k (increasing), backward for those before (decreasing),
// re-sampling the flow at each visited position.  Positions at reference r go
// to (px[r], py[r]).  Returns false if the event is masked: non-finite input,
// t outside [0,1], start off the image, or any visited position off the image.
template <int RM>
__device__ __forceinline__ bool warp_event(const WinParams& P, const Motion& m,
                                           const float* __restrict__ rho, double x0, double y0,
                                           double tk, double (&px)[RM], double (&py)[RM],
                                           int& mbefore)
{
    mbefore = 0;
    if (!(isfinite(x0) && isfinite(y0) && tk >= 0.0 && tk <= 1.0 && inside(P, x0, y0)))
        return false;
    const int mb = refs_before(P, tk);
    mbefore = mb;
    int r = mb;
    if (r < P.R && P.refs[r] == tk) {
        put(px, r, x0);
        put(py, r, y0);
        ++r;
    }
    // forward sweep
    double X = x0, Y = y0, tau = tk;
    for (; r < P.R; ++r) {
        double ux, uy;
        sample_flow(P, m, rho, X, Y, ux, uy);
        const double ref = P.refs[r];
        const double dt = ref - tau;
        X = X + dt * ux;
        Y = Y + dt * uy;
        tau = ref;
        if (!inside(P, X, Y)) return false;
        put(px, r, X);
        put(py, r, Y);
    }
    // backward sweep
    X = x0;
    Y = y0;
    tau = tk;
    for (r = mb - 1; r >= 0; --r) {
        double ux, uy;
        sample_flow(P, m, rho, X, Y, ux, uy);
        const double ref = P.refs[r];
        const double dt = ref - tau;
        X = X + dt * ux;
        Y = Y + dt * uy;
        tau = ref;
        if (!inside(P, X, Y)) return false;
        put(px, r, X);
        put(py, r, Y);
    }
    return true;
}

// Block-wide sum of doubles (blockDim.x a multiple of 64, <= 1024).
__device__ __forceinline__ double block_sum(double v, double* lds /* >= 16 */)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) lds[wid] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0) {
        const int nw = blockDim.x >> 6;
        for (int w = 0; w < nw; ++w) s += lds[w];
    }
    return s;   // valid in thread 0
}

}  // namespace cm
