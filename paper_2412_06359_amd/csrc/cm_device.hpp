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
// reference.  The splat images are FP64 as well (see cm_kernels.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace cm {

constexpr int kMaxRefs = 16;

constexpr int kMaxFlows = kMaxRefs + 1;   // segments between knots {0, 1} U refs

// Per-window constants, built on the host from the descriptor.
//
// Flow sets (Sec. 3.1 concatenates the flows of consecutive slices): a window
// warps with one flow (F = 1) or with one flow per segment between
// consecutive knots {0, 1} U refs, each from its own inverse depth
// (rho + f HW) and ego-motion (ego + 6 f).  A step that ends at reference r
// crosses the segment ending at r's knot when it runs forward in time
// (set sf[r]) and the segment starting there when it runs backward (sb[r]).
struct WinParams {
    int W, H, R, HW;
    int F;                      // flow sets
    int model;                  // flow model: 0 first-order motion field, 1 exact reprojection
    double cx, cy, fx, fy;
    double inv_fx, inv_fy, fx_over_fy, fy_over_fx;
    double xmax, ymax;          // W - 1, H - 1
    double eps;
    double two_over_R;
    double refs[kMaxRefs];
    int8_t sf[kMaxRefs], sb[kMaxRefs];
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

__device__ __forceinline__ Taps make_taps_wh(int W, int H, double X, double Y)
{
    Taps t;
    const double fx0 = floor(X), fy0 = floor(Y);
    t.x0 = (int)fx0;
    t.y0 = (int)fy0;
    t.a = X - fx0;
    t.b = Y - fy0;
    t.inx = t.x0 + 1 < W;
    t.iny = t.y0 + 1 < H;
    return t;
}

__device__ __forceinline__ Taps make_taps(const WinParams& P, double X, double Y)
{
    return make_taps_wh(P.W, P.H, X, Y);
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

// Offsets of the four taps from tap 0 for gathers that load every tap
// unconditionally: a tap off the sensor (not tap_in) reads its on-sensor
// neighbour instead, and the caller discards that value.  The four loads then
// carry no branch and issue back to back under one wait, where a load guarded
// by its tap_in test would pay a full memory latency per tap.
__device__ __forceinline__ void tap_offsets(const WinParams& P, const Taps& t, int (&off)[4])
{
    const int dx = t.inx ? 1 : 0, dy = t.iny ? P.W : 0;
    off[0] = 0;
    off[1] = dx;
    off[2] = dy;
    off[3] = dx + dy;
}

// Where the warp reads the flow: inverse depth and the motion coefficients.
// The flow at a tap, u = A + rho B, is recomputed in FP64 from rho (4 bytes a
// pixel, small enough to stay in L2) rather than read from a materialised FP64
// flow field (16 bytes a pixel), which measured slower.
struct FlowSrc {
    const float* __restrict__ rho;
    Motion m;
};

__device__ __forceinline__ FlowSrc flow_src(const WinParams& P, const float* __restrict__ rho,
                                            const float* __restrict__ ego)
{
    FlowSrc f;
    f.rho = rho;
    f.m = load_motion(P, ego);
    return f;
}

// ---------------------------------------------------------------------------
// Exact reprojection (Eq. 2 without the first-order expansion).  The pixel's
// ray xn = ((i - cx)/fx, (j - cy)/fy, 1) at inverse depth rho is the point
// xn/rho; the pose maps it to R xn/rho + v, which projects like
//   p = R xn + rho v,   u = (fx p_x/p_z + cx - i, fy p_y/p_z + cy - j);
// a point on or behind the camera plane (p_z <= 0) gets zero flow.
//
// R = I + a K + b K^2 and the right Jacobian of the exponential map
// Jr = I - b K + c K^2 (K = [w]x, t = |w|) use a = sin t/t, b = (1 - cos t)/t^2,
// c = (t - sin t)/t^3, evaluated as their power series in t^2 (Horner, 18
// terms: below 1e-16 relative for t <= pi), so that every operation is plain
// FP64 arithmetic in a fixed order.
// ---------------------------------------------------------------------------
struct MotionX {
    double R[9];     // row-major rotation
    double v[3];     // translation
};

struct MotionXJ {
    double R[9];
    double v[3];
    double Jr[9];    // right Jacobian, row-major
};

// sum_k (-s)^k / ((2k+o)! / o!) ... with o the first denominator offset:
// series(s, o) = 1 - s/((o+1)(o+2)) (1 - s/((o+3)(o+4)) (1 - ...)).
__device__ __forceinline__ double rot_series(double s, int o)
{
    double h = 1.0;
#pragma unroll
    for (int k = 18; k >= 1; --k) {
        const double d = (double)(o + 2 * k - 1) * (double)(o + 2 * k);
        h = 1.0 - (s / d) * h;
    }
    return h;
}

__device__ __forceinline__ void rotation_exp(double wx, double wy, double wz, double (&R)[9],
                                             double* Jr)
{
    const double s = (wx * wx + wy * wy) + wz * wz;
    const double a = rot_series(s, 1);           // sin t / t
    const double b = 0.5 * rot_series(s, 2);     // (1 - cos t) / t^2
    const double K[9] = {0.0, -wz, wy, wz, 0.0, -wx, -wy, wx, 0.0};
    double K2[9];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j)
            K2[3 * i + j] = (K[3 * i + 0] * K[0 * 3 + j] + K[3 * i + 1] * K[1 * 3 + j]) +
                            K[3 * i + 2] * K[2 * 3 + j];
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        const double I = (i % 4 == 0) ? 1.0 : 0.0;
        R[i] = (I + a * K[i]) + b * K2[i];
    }
    if (Jr) {
        const double c = rot_series(s, 3) / 6.0;   // (t - sin t) / t^3
#pragma unroll
        for (int i = 0; i < 9; ++i) {
            const double I = (i % 4 == 0) ? 1.0 : 0.0;
            Jr[i] = (I - b * K[i]) + c * K2[i];
        }
    }
}

__device__ __forceinline__ void rotation_of(const float* __restrict__ ego, double (&R)[9],
                                            double* Jr)
{
    rotation_exp(ego[3], ego[4], ego[5], R, Jr);
}

__device__ __forceinline__ MotionX load_motion_x(const float* __restrict__ ego)
{
    MotionX m;
    rotation_of(ego, m.R, nullptr);
    m.v[0] = ego[0];
    m.v[1] = ego[1];
    m.v[2] = ego[2];
    return m;
}

__device__ __forceinline__ MotionXJ load_motion_xj(const float* __restrict__ ego)
{
    MotionXJ m;
    rotation_of(ego, m.R, m.Jr);
    m.v[0] = ego[0];
    m.v[1] = ego[1];
    m.v[2] = ego[2];
    return m;
}

// Where the warp reads an exact flow: inverse depth and the set's pose.
struct FlowSrcX {
    const float* __restrict__ rho;
    const MotionX* m;
};

// The flows of a window, by set.  FM (flow kind) 0: one first-order flow in
// registers; 1: first-order flows, motion coefficients in a per-block LDS
// table; 2: exact-reprojection flows, poses in the LDS table.  Set f reads
// inverse depth at rho + f HW.
union MotionTable {
    Motion m[kMaxFlows];
    MotionX x[kMaxFlows];
};

template <int FM>
struct Flows;

template <>
struct Flows<0> {
    FlowSrc f;
    __device__ __forceinline__ const FlowSrc& at(int) const { return f; }
};

template <>
struct Flows<1> {
    const float* __restrict__ rho;
    int HW;
    const Motion* m;
    __device__ __forceinline__ FlowSrc at(int s) const
    {
        FlowSrc f;
        f.rho = rho + (size_t)s * HW;
        f.m = m[s];
        return f;
    }
};

template <>
struct Flows<2> {
    const float* __restrict__ rho;
    int HW;
    const MotionX* m;
    __device__ __forceinline__ FlowSrcX at(int s) const
    {
        FlowSrcX f;
        f.rho = rho + (size_t)s * HW;
        f.m = m + s;
        return f;
    }
};

// Builds a block's flows.  `mt` is the block's LDS table (used with FM 1, 2);
// all threads call this, followed by a barrier before the first use.
template <int FM>
__device__ __forceinline__ Flows<FM> make_flows(const WinParams& P, const float* __restrict__ rho,
                                                const float* __restrict__ ego, MotionTable* mt);

template <>
__device__ __forceinline__ Flows<0> make_flows<0>(const WinParams& P,
                                                  const float* __restrict__ rho,
                                                  const float* __restrict__ ego, MotionTable*)
{
    Flows<0> fl;
    fl.f = flow_src(P, rho, ego);
    return fl;
}

template <>
__device__ __forceinline__ Flows<1> make_flows<1>(const WinParams& P,
                                                  const float* __restrict__ rho,
                                                  const float* __restrict__ ego, MotionTable* mt)
{
    if ((int)threadIdx.x < P.F) mt->m[threadIdx.x] = load_motion(P, ego + 6 * threadIdx.x);
    Flows<1> fl;
    fl.rho = rho;
    fl.HW = P.HW;
    fl.m = mt->m;
    return fl;
}

template <>
__device__ __forceinline__ Flows<2> make_flows<2>(const WinParams& P,
                                                  const float* __restrict__ rho,
                                                  const float* __restrict__ ego, MotionTable* mt)
{
    if ((int)threadIdx.x < P.F) mt->x[threadIdx.x] = load_motion_x(ego + 6 * threadIdx.x);
    Flows<2> fl;
    fl.rho = rho;
    fl.HW = P.HW;
    fl.m = mt->x;
    return fl;
}

// As make_flows, with one flow's motion coefficients read from a per-set
// table in device memory: the address is uniform over the block, so the
// coefficients stay in scalar registers instead of occupying vector registers
// for the whole kernel.
template <int FM>
__device__ __forceinline__ Flows<FM> make_flows_tab(const WinParams& P,
                                                    const float* __restrict__ rho,
                                                    const float* __restrict__ ego,
                                                    const Motion* __restrict__ mtab,
                                                    MotionTable* mt)
{
    if constexpr (FM == 0) {
        Flows<0> fl;
        fl.f.rho = rho;
        fl.f.m = mtab[0];
        return fl;
    } else {
        return make_flows<FM>(P, rho, ego, mt);
    }
}

__device__ __forceinline__ double2 flow_at(const WinParams& P, const Motion& m, int i, int j,
                                           double r)
{
    double Ax, Ay, Bx, By;
    flow_parts(P, m, i, j, Ax, Ay, Bx, By);
    return make_double2(Ax + r * Bx, Ay + r * By);
}

// The flow at the four taps of a position on the image (zero off the sensor).
// The taps share two columns and two rows, so the terms that depend on one
// coordinate only are formed once per column or row; every value is the same
// FP64 operation as flow_parts on that tap.
__device__ __forceinline__ void tap_flows(const WinParams& P, const FlowSrc& f, const Taps& t,
                                          double2 (&uq)[4])
{
    const Motion& m = f.m;
    const double xb[2] = {(double)t.x0 - P.cx, (double)(t.x0 + 1) - P.cx};
    const double yb[2] = {(double)t.y0 - P.cy, (double)(t.y0 + 1) - P.cy};
    double k3x[2], k2y[2], cy[2], dx[2], Bx[2], By[2];
#pragma unroll
    for (int i = 0; i < 2; ++i) {
        k3x[i] = m.k3 * xb[i];
        k2y[i] = m.k2 * yb[i];
        cy[i] = m.k0 - m.k1 * yb[i];
        dx[i] = m.k4 + m.k5 * xb[i];
        Bx[i] = m.tvx - xb[i] * m.vz;
        By[i] = m.tvy - yb[i] * m.vz;
    }
    const float* row0 = f.rho + (size_t)t.y0 * P.W + t.x0;
    int off[4];
    tap_offsets(P, t, off);
    float rq[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) rq[q] = row0[off[q]];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int a = q & 1, b = q >> 1;
        const double s = k3x[a] - k2y[b];
        const double Ax = cy[b] + xb[a] * s;
        const double Ay = dx[a] + yb[b] * s;
        const double r = (double)rq[q];
        uq[q] = tap_in(t, q) ? make_double2(Ax + r * Bx[a], Ay + r * By[b])
                             : make_double2(0.0, 0.0);
    }
}

// The exact flow at the four taps; the row and column terms of R xn are formed
// once per column or row:  p_k = (R[k][0] xn + (R[k][1] yn + R[k][2])) + rho v_k.
__device__ __forceinline__ void tap_flows(const WinParams& P, const FlowSrcX& f, const Taps& t,
                                          double2 (&uq)[4])
{
    const MotionX& m = *f.m;
    double col[2][3], row[2][3];
#pragma unroll
    for (int a = 0; a < 2; ++a) {
        const double xn = ((double)(t.x0 + a) - P.cx) * P.inv_fx;
        const double yn = ((double)(t.y0 + a) - P.cy) * P.inv_fy;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            col[a][k] = m.R[3 * k + 0] * xn;
            row[a][k] = m.R[3 * k + 1] * yn + m.R[3 * k + 2];
        }
    }
    const float* row0 = f.rho + (size_t)t.y0 * P.W + t.x0;
    int off[4];
    tap_offsets(P, t, off);
    float rq[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) rq[q] = row0[off[q]];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int a = q & 1, b = q >> 1;
        const double r = (double)rq[q];
        const double px = (col[a][0] + row[b][0]) + r * m.v[0];
        const double py = (col[a][1] + row[b][1]) + r * m.v[1];
        const double pz = (col[a][2] + row[b][2]) + r * m.v[2];
        double2 u = make_double2(0.0, 0.0);
        if (tap_in(t, q) && pz > 0.0) {
            const double iz = 1.0 / pz;
            u.x = (P.fx * px) * iz + (P.cx - (double)(t.x0 + a));
            u.y = (P.fy * py) * iz + (P.cy - (double)(t.y0 + b));
        }
        uq[q] = u;
    }
}

// BS(u)(X, Y): the flow sampled bilinearly at a position on the image.  At a
// pixel centre (both fractional parts zero) taps 1-3 carry zero weight and
// only add signed zeros to the sum, so they are treated as off the sensor and
// their inverse depth is not loaded: events lie on pixel centres, and the
// warp's first sample of every event is taken there.
template <typename Src>
__device__ __forceinline__ void sample_flow(const WinParams& P, const Src& f, double X,
                                            double Y, double& ux, double& uy)
{
    Taps t = make_taps(P, X, Y);
    if (t.a == 0.0 && t.b == 0.0) {
        t.inx = false;
        t.iny = false;
    }
    double2 uq[4];
    tap_flows(P, f, t, uq);
    ux = 0.0;
    uy = 0.0;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const double w = tap_w(t, q);
        ux += w * uq[q].x;
        uy += w * uq[q].y;
    }
}

// Number of reference times strictly before t.
__device__ __forceinline__ int refs_before(const WinParams& P, double t)
{
    int m = 0;
#pragma unroll
    for (int r = 0; r < kMaxRefs; ++r) m += (r < P.R && P.refs[r] < t) ? 1 : 0;
    return m;
}

// Per-block table of the reference times and adjoint seed coefficients
// (2/R)/(N_r + eps), read with a per-lane index.
struct RefTable {
    double t[kMaxRefs];
    double coef[kMaxRefs];
    int sf[kMaxRefs], sb[kMaxRefs];   // flow set of the forward / backward step into r
};

// An event's visits of the reference times.  Visit j (0 <= j < R) is
// reference vr[j]: first the forward sweep over the references at or after
// t_k in increasing order (j < nf), then the backward sweep over those before
// t_k in decreasing order.  A reference equal to t_k is the first forward
// visit and keeps the event's position.
struct Visits {
    int nf;      // forward visits
    int mb;      // references before t_k (backward visits)
    bool eq;     // the first forward visit is a reference equal to t_k
};

// Sec. 3.1 / 3.3: push one event through the reference times, re-sampling the
// flow at each visited position; (vx[j], vy[j]) is the position at visit j.
// Returns false if the event is masked: non-finite input, t outside [0,1],
// start off the image, or any visited position off the image.  The loop is
// unrolled over visits so that every array index is static, and all lanes of a
// wave step through the same visit numbers together.
// The same warp handing each visit (j, X, Y, reference) to `visit` as it is
// reached instead of storing the positions (the mask still applies to the
// whole event: a false return discards what the visitor saw).
template <int RM, int FM, typename Visit>
__device__ __forceinline__ bool warp_visits_v(const WinParams& P, const Flows<FM>& fl,
                                              const RefTable& rt, double x0, double y0,
                                              double tk, Visits& v, Visit&& visit)
{
    v.nf = 0;
    v.mb = 0;
    v.eq = false;
    if (!(isfinite(x0) && isfinite(y0) && tk >= 0.0 && tk <= 1.0 && inside(P, x0, y0)))
        return false;
    const int mb = refs_before(P, tk);
    v.mb = mb;
    v.nf = P.R - mb;
    v.eq = v.nf > 0 && rt.t[mb] == tk;
    // Both sweeps start at the event; when their first steps use the same flow
    // (always with one flow set) the sample there is taken once.
    double u0x = 0.0, u0y = 0.0;
    int u0set = -1;
    double X = x0, Y = y0, tau = tk;
    bool at_event = true;
#pragma unroll
    for (int j = 0; j < RM; ++j) {
        if (j < P.R) {
            int r, set;
            if (j < v.nf) {
                r = mb + j;
                set = FM ? rt.sf[r] : 0;
            } else {
                r = mb - 1 - (j - v.nf);
                set = FM ? rt.sb[r] : 0;
                if (j == v.nf) {
                    X = x0;
                    Y = y0;
                    tau = tk;
                    at_event = true;
                }
            }
            const double ref = rt.t[r];
            const double dt = ref - tau;
            if (dt != 0.0) {
                double ux = u0x, uy = u0y;
                if (!(at_event && u0set == set)) {
                    sample_flow(P, fl.at(set), X, Y, ux, uy);
                    if (at_event) {
                        u0x = ux;
                        u0y = uy;
                        u0set = set;
                    }
                }
                X = X + dt * ux;
                Y = Y + dt * uy;
                at_event = false;
            }
            tau = ref;
            if (!inside(P, X, Y)) return false;
            visit(j, X, Y, r);
        }
    }
    return true;
}

template <int RM, int FM>
__device__ __forceinline__ bool warp_visits(const WinParams& P, const Flows<FM>& fl,
                                            const RefTable& rt, double x0, double y0, double tk,
                                            double (&vx)[RM], double (&vy)[RM], int (&vr)[RM],
                                            Visits& v)
{
    return warp_visits_v<RM, FM>(P, fl, rt, x0, y0, tk, v, [&](int j, double X, double Y, int r) {
        vx[j] = X;
        vy[j] = Y;
        vr[j] = r;
    });
}

// The warp step that ends at visit j: whether it is a real step (not the
// reference equal to t_k), whether it starts at the event (the first step of
// its sweep), and its dt.  The reverse pass walks j = R-1 .. 0 (the backward
// sweep backwards, then the forward sweep backwards), restarting the adjoint
// at j = R-1 and at j = nf-1.
struct VisitStep {
    bool step, first, restart;
    int set;        // flow set of the step
    double dt;
};

// The reference of visit j: mb + j in the forward sweep, mb - 1 - (j - nf)
// in the backward sweep (the same order warp_visits_v takes).
__device__ __forceinline__ int visit_ref(const Visits& v, int j)
{
    return j < v.nf ? v.mb + j : v.mb - 1 - (j - v.nf);
}

__device__ __forceinline__ VisitStep visit_step(const WinParams& P, const RefTable& rt,
                                                const Visits& v, int j, double tk)
{
    VisitStep s;
    const int jf = v.eq ? 1 : 0;             // first real forward step
    const int r = visit_ref(v, j);
    s.step = !(v.eq && j == 0);
    s.first = (j == jf && j < v.nf) || (j == v.nf);
    s.restart = (j == P.R - 1) || (j == v.nf - 1);
    const double tprev = (s.first || j == 0) ? tk : rt.t[visit_ref(v, j > 0 ? j - 1 : 0)];
    s.dt = rt.t[r] - tprev;
    s.set = (j < v.nf) ? rt.sf[r] : rt.sb[r];
    return s;
}

// Direct sensitivity of the loss to the position of an event on reference r:
// sum over taps of (dL/dC + tbar dL/dS) grad w, with
//   dL/dS = coef S/(C+eps)^2,  dL/dC = -coef S^2/(C+eps)^3,  coef = (2/R)/(N_r+eps).
__device__ __forceinline__ void direct_term(const WinParams& P, const double2* __restrict__ plane,
                                            double coef, double tb, double X, double Y,
                                            double& Lx, double& Ly)
{
    const Taps tp = make_taps(P, X, Y);
    int off[4];
    tap_offsets(P, tp, off);
    const double2* p0 = plane + tap_pix(P, tp, 0);
    double2 csq[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) csq[q] = p0[off[q]];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        if (!tap_in(tp, q)) continue;
        const double2 cs = csq[q];
        const double S = cs.y;
        const double inv = 1.0 / (cs.x + P.eps);
        const double sc = S * inv;
        const double g = coef * sc * inv * (tb - sc);
        double dX, dY;
        tap_dw(tp, q, dX, dY);
        Lx += g * dX;
        Ly += g * dY;
    }
}

// d theta contribution of dL/du = (gx, gy) at pixel (i, j) with inverse depth
// r: the transpose of d u / d theta (first-order Eq. 2) applied to g.
__device__ __forceinline__ void dtheta_at_pixel(const WinParams& P, int i, int j, double r,
                                                double gx, double gy, double (&dth)[6])
{
    const double xb = (double)i - P.cx, yb = (double)j - P.cy;
    dth[0] += r * P.fx * gx;
    dth[1] += r * P.fy * gy;
    dth[2] -= r * (xb * gx + yb * gy);
    dth[3] -= (xb * yb * P.inv_fy) * gx + (P.fy + yb * yb * P.inv_fy) * gy;
    dth[4] += (P.fx + xb * xb * P.inv_fx) * gx + (xb * yb * P.inv_fx) * gy;
    dth[5] += (P.fy_over_fx * xb) * gy - (P.fx_over_fy * yb) * gx;
}

// Exact model: d rho and d theta of dL/du = (gx, gy) at pixel (i, j) with
// inverse depth r.  With J = du/dp = [[fx/pz, 0, -fx px/pz^2], [0, fy/pz,
// -fy py/pz^2]] and q = J^T g:  d rho = q . v,  d v += r q,
// d w += Jr^T (xn x (R^T q))  (the adjoint of d(R xn)/dw = -R [xn]x Jr).
// Returns d rho (zero for a point on or behind the camera plane).
__device__ __forceinline__ double chain_exact(const WinParams& P, const MotionXJ& m, int i, int j,
                                              double r, double gx, double gy, double (&dth)[6])
{
    const double xn = ((double)i - P.cx) * P.inv_fx;
    const double yn = ((double)j - P.cy) * P.inv_fy;
    double p[3];
#pragma unroll
    for (int k = 0; k < 3; ++k)
        p[k] = (m.R[3 * k + 0] * xn + (m.R[3 * k + 1] * yn + m.R[3 * k + 2])) + r * m.v[k];
    if (!(p[2] > 0.0)) return 0.0;
    const double iz = 1.0 / p[2];
    const double ax = gx * P.fx, ay = gy * P.fy;
    const double q[3] = {ax * iz, ay * iz, -((ax * p[0] + ay * p[1]) * iz) * iz};
    const double drho = (q[0] * m.v[0] + q[1] * m.v[1]) + q[2] * m.v[2];
#pragma unroll
    for (int k = 0; k < 3; ++k) dth[k] += r * q[k];
    double sv[3];
#pragma unroll
    for (int k = 0; k < 3; ++k)
        sv[k] = (m.R[0 * 3 + k] * q[0] + m.R[1 * 3 + k] * q[1]) + m.R[2 * 3 + k] * q[2];
    const double cr[3] = {yn * sv[2] - sv[1], sv[0] - xn * sv[2], xn * sv[1] - yn * sv[0]};
#pragma unroll
    for (int k = 0; k < 3; ++k)
        dth[3 + k] += (m.Jr[0 * 3 + k] * cr[0] + m.Jr[1 * 3 + k] * cr[1]) + m.Jr[2 * 3 + k] * cr[2];
    return drho;
}

// J(P)^T L for the bilinear flow sample at (X, Y): sum over taps of
// (L . u_tap) grad w_tap.
template <typename Src>
__device__ __forceinline__ void jacobian_t(const WinParams& P, const Src& u,
                                           double X, double Y, double Lx, double Ly, double& jx,
                                           double& jy)
{
    const Taps tp = make_taps(P, X, Y);
    double2 uq[4];
    tap_flows(P, u, tp, uq);
    jx = 0.0;
    jy = 0.0;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const double lu = Lx * uq[q].x + Ly * uq[q].y;
        double dX, dY;
        tap_dw(tp, q, dX, dY);
        jx += lu * dX;
        jy += lu * dY;
    }
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

// K block_sum reductions in one pass: each value is added up in block_sum's
// order, with one pair of barriers for all of them.  Results in thread 0.
// nwaves (default: all of the block's) is the number of leading wavefronts
// whose values count, as if the block had only those.
template <int K>
__device__ __forceinline__ void block_sum_n(double (&v)[K], double* lds /* >= 16 K */,
                                            int nwaves = 0)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1)
#pragma unroll
        for (int k = 0; k < K; ++k) v[k] += __shfl_down(v[k], o, 64);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0)
#pragma unroll
        for (int k = 0; k < K; ++k) lds[16 * k + wid] = v[k];
    __syncthreads();
    if (threadIdx.x == 0) {
        const int nw = nwaves > 0 ? nwaves : (int)(blockDim.x >> 6);
#pragma unroll
        for (int k = 0; k < K; ++k) {
            double s = 0.0;
            for (int w = 0; w < nw; ++w) s += lds[16 * k + w];
            v[k] = s;
        }
    }
}

}  // namespace cm

namespace cm {

// ---------------------------------------------------------------------------
// Tiled (owner-computes) splat geometry.  The image is cut into TW x TH tiles;
// a warped position belongs to the tile of its tap (x0, y0), so its taps fall
// in that tile or in the tile's right column / bottom row halo.
// ---------------------------------------------------------------------------
constexpr int TW = 32, TH = 32;
constexpr int TLW = TW + 1, TLH = TH + 1;    // LDS tile with halo
constexpr int NHALO = TH + 1 + TW;           // right column (rows 0..TH) + bottom row (cols 0..TW-1)
constexpr int NBORDER = TW + TH - 1;         // own column 0 (rows 0..TH-1) + row 0 (cols 1..TW-1)
constexpr int kMaxBins = 16384;              // LDS histogram limit (64 KB)
constexpr int kBinThreads = 256;             // threads of the count / scatter kernels
constexpr int kMaxEventsPerThread = 16;


struct TileGeom {
    int tw, th;             // tile size (powers of two; 32 x 32 in the deterministic mode)
    int tws, ths;           // their base-2 logarithms
    int ntx, nty, ntiles;   // tiles per row / column / image
    int nbins;              // forward bins: R * ntiles (reference, tile)
    int nbins_b;            // backward bins: F * ntiles (flow set, tile)
    int nbins_s;            // source-record bins (atomic mode): ntiles; 0 otherwise
    int nblocks;            // count / scatter blocks
    int ept;                // events per thread in the count / scatter kernels
};

// Forward record: a warped position on one reference time.
struct SplatRec {
    double X, Y;
    float ts;               // event time, sign bit = polarity (set: negative)
    uint32_t k;             // event index
};

// A valid event as the backward reads it: coordinates, time with the
// polarity in the sign bit (set: negative), index.  The forward writes one per
// valid event in the order of its reference-0 splat records (grouped by the
// tile its reference-0 position falls in), so that neighbouring lanes of the
// backward warp, sample and gather near each other.
struct SrcRec {
    float x0, y0, ts;
    uint32_t k;
};

// Backward record: a warp step's sampling position and dt * adjoint.
struct GradRec {
    double X, Y;
    double gx, gy;
};

// Record I/O with the non-temporal hint: each record is written once and read
// once, so the stream of records should not push the inverse-depth and image
// lines that the gathers reuse out of the caches.
typedef double nt_d2 __attribute__((ext_vector_type(2), aligned(8)));
typedef uint32_t nt_u2 __attribute__((ext_vector_type(2), aligned(8)));
typedef uint32_t nt_u4 __attribute__((ext_vector_type(4), aligned(16)));

__device__ __forceinline__ void store_nt(SplatRec* p, const SplatRec& q)
{
    const nt_d2 a = {q.X, q.Y};
    const nt_u2 b = {__float_as_uint(q.ts), q.k};
    __builtin_nontemporal_store(a, reinterpret_cast<nt_d2*>(p));
    __builtin_nontemporal_store(b, reinterpret_cast<nt_u2*>(reinterpret_cast<char*>(p) + 16));
}

__device__ __forceinline__ SplatRec load_nt(const SplatRec* p)
{
    const nt_d2 a = __builtin_nontemporal_load(reinterpret_cast<const nt_d2*>(p));
    const nt_u2 b = __builtin_nontemporal_load(
        reinterpret_cast<const nt_u2*>(reinterpret_cast<const char*>(p) + 16));
    SplatRec q;
    q.X = a.x;
    q.Y = a.y;
    q.ts = __uint_as_float(b.x);
    q.k = b.y;
    return q;
}

// An event-sampled backward record: dt * adjoint at the event, whose
// position its source record holds (16 bytes at the source record's index).
__device__ __forceinline__ void store_nt(double2* p, double gx, double gy)
{
    const nt_d2 a = {gx, gy};
    __builtin_nontemporal_store(a, reinterpret_cast<nt_d2*>(p));
}

__device__ __forceinline__ double2 load_nt(const double2* p)
{
    const nt_d2 a = __builtin_nontemporal_load(reinterpret_cast<const nt_d2*>(p));
    return make_double2(a.x, a.y);
}

__device__ __forceinline__ void store_nt(GradRec* p, const GradRec& q)
{
    const nt_d2 a = {q.X, q.Y}, b = {q.gx, q.gy};
    __builtin_nontemporal_store(a, reinterpret_cast<nt_d2*>(p));
    __builtin_nontemporal_store(b, reinterpret_cast<nt_d2*>(p) + 1);
}

__device__ __forceinline__ GradRec load_nt(const GradRec* p)
{
    const nt_d2 a = __builtin_nontemporal_load(reinterpret_cast<const nt_d2*>(p));
    const nt_d2 b = __builtin_nontemporal_load(reinterpret_cast<const nt_d2*>(p) + 1);
    GradRec q;
    q.X = a.x;
    q.Y = a.y;
    q.gx = b.x;
    q.gy = b.y;
    return q;
}

__device__ __forceinline__ void store_nt(SrcRec* p, const SrcRec& q)
{
    const nt_u4 a = {__float_as_uint(q.x0), __float_as_uint(q.y0), __float_as_uint(q.ts), q.k};
    __builtin_nontemporal_store(a, reinterpret_cast<nt_u4*>(p));
}

__device__ __forceinline__ SrcRec load_nt(const SrcRec* p)
{
    const nt_u4 a = __builtin_nontemporal_load(reinterpret_cast<const nt_u4*>(p));
    SrcRec q;
    q.x0 = __uint_as_float(a.x);
    q.y0 = __uint_as_float(a.y);
    q.ts = __uint_as_float(a.z);
    q.k = a.w;
    return q;
}

__device__ __forceinline__ int tile_index(const TileGeom& G, const Taps& t)
{
    return (int)((uint32_t)t.y0 >> G.ths) * G.ntx + (int)((uint32_t)t.x0 >> G.tws);
}

// The tiles whose pixels the on-sensor taps of a position reach (atomic
// mode, where each tile owns all its pixels): the tile of tap 0 and, when tap
// 0 sits on that tile's last column or row, the right, lower and lower-right
// neighbours.  Packed as the tile index (low 16 bits) and two flags: bit 16,
// the right neighbour is reached; bit 17, the lower one (both: the
// lower-right one as well).  A tap of zero weight counts: the backward reads
// the image at every tap of a position, so its pixel must be stored.
constexpr uint32_t kReachRight = 1u << 16, kReachDown = 1u << 17;

__device__ __forceinline__ uint32_t tiles_reached(const TileGeom& G, const Taps& t)
{
    const uint32_t x0 = (uint32_t)t.x0, y0 = (uint32_t)t.y0;
    uint32_t v = (uint32_t)((y0 >> G.ths) * G.ntx + (x0 >> G.tws));
    if (t.inx && (x0 & (G.tw - 1)) == (uint32_t)G.tw - 1) v |= kReachRight;
    if (t.iny && (y0 & (G.th - 1)) == (uint32_t)G.th - 1) v |= kReachDown;
    return v;
}

// Calls fn(tile) for every tile of a packed tiles_reached value, own tile first.
template <typename F>
__device__ __forceinline__ void for_each_reached(uint32_t v, int ntx, F&& fn)
{
    const int tile = (int)(v & 0xffffu);
    fn(tile);
    if (v & kReachRight) fn(tile + 1);
    if (v & kReachDown) fn(tile + ntx);
    if ((v & kReachRight) && (v & kReachDown)) fn(tile + ntx + 1);
}

}  // namespace cm
