// cm_kernels.hip -- HIP kernels of the CM loss for gfx950 (single window).
//
//   fill_zero          clears the splat images and per-window sums
//   splat_kernel       per event: iterative warp (FP64) + bilinear splat into
//                      the per-polarity images C and S with FP64 global
//                      atomics (paper Sec. 3.1, Fig. 2; Sec. 3.3 per-event
//                      forward)
//   reduce_kernel      per reference: sum_x sum_p (S_p/(C_p+eps))^2 and the
//                      active-pixel count (Eq. 1), FP64 block partials
//   finalize_forward   fixed-order sum of the partials, mean over references
//   backward_kernel    per event: recompute the warp, gather the adjoint seeds
//                      at the splat taps, reverse sweep through the warp
//                      steps, FP32 atomics into d rho, FP64 block partials of
//                      d theta (Sec. 3.3 analytic backward)
//   finalize_backward  fixed-order sum of the d theta partials
//
// State image layout (FP64): img[((r * 2 + pol) * H * W + pix) * 2 + ch],
// pol 0 = positive, 1 = negative; ch 0 = C (weights), ch 1 = S (weights times
// the timestamp contribution).  C and S of one pixel share 16 bytes, and the two
// horizontally adjacent taps of an event share 32 bytes.
//
// The images are FP64 because the adjoint seed (t_k - S/(C+eps)) cancels at
// pixels that one event dominates: there S/(C+eps) equals t_k up to terms of
// order eps/C, and FP32 rounding of C and S (relative 6e-8) swamps them when C
// is a small bilinear weight.
#include "cm_kernels.hpp"

namespace cm {

__global__ __launch_bounds__(256) void fill_zero_kernel(float* __restrict__ p, size_t n,
                                                        int vec4)
{
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    const size_t tid = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (vec4) {
        float4* p4 = reinterpret_cast<float4*>(p);
        const size_t n4 = n / 4;
        const float4 z = make_float4(0.f, 0.f, 0.f, 0.f);
        for (size_t i = tid; i < n4; i += stride) p4[i] = z;
        for (size_t i = n4 * 4 + tid; i < n; i += stride) p[i] = 0.f;
    } else {
        for (size_t i = tid; i < n; i += stride) p[i] = 0.f;
    }
}

template <int RM, int FM>
__global__ __launch_bounds__(256) void splat_kernel(WinParams P, const float* __restrict__ ex,
                                                    const float* __restrict__ ey,
                                                    const float* __restrict__ et,
                                                    const int8_t* __restrict__ ep, int64_t n,
                                                    const float* __restrict__ rho,
                                                    const float* __restrict__ ego,
                                                    double* __restrict__ img,
                                                    unsigned long long* __restrict__ n_valid)
{
    __shared__ unsigned int cnt_lds;
    __shared__ RefTable rt;
    __shared__ MotionTable mt;
    if (threadIdx.x == 0) cnt_lds = 0;
    if (threadIdx.x < kMaxRefs) {
        rt.t[threadIdx.x] = P.refs[threadIdx.x];
        rt.sf[threadIdx.x] = P.sf[threadIdx.x];
        rt.sb[threadIdx.x] = P.sb[threadIdx.x];
    }
    const Flows<FM> u = make_flows<FM>(P, rho, ego, &mt);
    __syncthreads();
    unsigned int cnt = 0;
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n;
         k += (int64_t)gridDim.x * blockDim.x) {
        const double x0 = ex[k], y0 = ey[k], tk = et[k];
        const int pol = ep[k] > 0 ? 0 : 1;
        double vx[RM], vy[RM];
        int vr[RM];
        Visits v;
        if (!warp_visits<RM, FM>(P, u, rt, x0, y0, tk, vx, vy, vr, v)) continue;
        ++cnt;
#pragma unroll
        for (int j = 0; j < RM; ++j) {
            if (j < P.R) {
                const int r = vr[j];
                const Taps tp = make_taps(P, vx[j], vy[j]);
                const double tb = 1.0 - fabs(rt.t[r] - tk);
                double* plane = img + (size_t)(r * 2 + pol) * P.HW * 2;
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    if (!tap_in(tp, q)) continue;
                    const double w = tap_w(tp, q);
                    if (w == 0.0) continue;
                    const int pix = tap_pix(P, tp, q);
                    unsafeAtomicAdd(plane + 2 * pix, w);
                    unsafeAtomicAdd(plane + 2 * pix + 1, w * tb);
                }
            }
        }
    }
    if (cnt) atomicAdd(&cnt_lds, cnt);
    __syncthreads();
    if (threadIdx.x == 0 && cnt_lds) atomicAdd(n_valid, (unsigned long long)cnt_lds);
}

__global__ __launch_bounds__(256) void reduce_kernel(WinParams P, const double* __restrict__ img,
                                                     double* __restrict__ part, int RB)
{
    __shared__ double lds[16];
    const int r = blockIdx.y;
    const double2* Cp = reinterpret_cast<const double2*>(img) + (size_t)(r * 2 + 0) * P.HW;
    const double2* Cm = reinterpret_cast<const double2*>(img) + (size_t)(r * 2 + 1) * P.HW;
    double sum = 0.0, cnt = 0.0;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < P.HW; i += RB * blockDim.x) {
        const double2 a = Cp[i], b = Cm[i];
        if (a.x + b.x > 0.0) cnt += 1.0;
        if (a.x != 0.0 || a.y != 0.0) {
            const double T = a.y / (a.x + P.eps);
            sum += T * T;
        }
        if (b.x != 0.0 || b.y != 0.0) {
            const double T = b.y / (b.x + P.eps);
            sum += T * T;
        }
    }
    const double s = block_sum(sum, lds);
    const double c = block_sum(cnt, lds);
    if (threadIdx.x == 0) {
        part[((size_t)r * RB + blockIdx.x) * 2 + 0] = s;
        part[((size_t)r * RB + blockIdx.x) * 2 + 1] = c;
    }
}

__global__ __launch_bounds__(256) void finalize_forward_kernel(WinParams P,
                                                               const double* __restrict__ part,
                                                               int RB, StateHeader* hdr,
                                                               float* __restrict__ loss)
{
    __shared__ double lds[16];
    double L = 0.0;
    for (int r = 0; r < P.R; ++r) {
        double s = 0.0, c = 0.0;
        for (int b = threadIdx.x; b < RB; b += blockDim.x) {
            s += part[((size_t)r * RB + b) * 2 + 0];
            c += part[((size_t)r * RB + b) * 2 + 1];
        }
        s = block_sum(s, lds);
        c = block_sum(c, lds);
        if (threadIdx.x == 0) {
            hdr->num[r] = s;
            hdr->nact[r] = c;
            L += s / (c + P.eps);
        }
    }
    if (threadIdx.x == 0) {
        L = L / (double)P.R;
        hdr->loss = L;
        loss[0] = (float)L;
    }
}

// Adjoint of one warp step P_j = P_{j-1} + dt BS(u)(P_{j-1}) at P_{j-1} = (X, Y):
// scatters dL/du at the taps into d rho (through du/drho = B) and d theta,
// and advances the adjoint (Lx, Ly) <- L + dt J^T L.
__device__ __forceinline__ void adjoint_step(const WinParams& P, const FlowSrc& u, double X,
                                             double Y,
                                             double dt, double& Lx, double& Ly, double gl,
                                             float* __restrict__ drho, double (&dth)[6])
{
    const Taps tp = make_taps(P, X, Y);
    double2 uq[4];
    tap_flows(P, u, tp, uq);
    double jx = 0.0, jy = 0.0;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        double dX, dY;
        tap_dw(tp, q, dX, dY);
        const double lu = Lx * uq[q].x + Ly * uq[q].y;
        jx += lu * dX;
        jy += lu * dY;
        if (!tap_in(tp, q)) continue;
        const double w = tap_w(tp, q);
        if (w != 0.0) {
            const int i = tp.x0 + (q & 1), j = tp.y0 + (q >> 1);
            const int pix = j * P.W + i;
            double Ax, Ay, Bx, By;
            flow_parts(P, u.m, i, j, Ax, Ay, Bx, By);
            const double gx = dt * w * Lx, gy = dt * w * Ly;
            unsafeAtomicAdd(drho + pix, (float)(gl * (gx * Bx + gy * By)));
            dtheta_at_pixel(P, i, j, (double)u.rho[pix], gx, gy, dth);
        }
    }
    Lx += dt * jx;
    Ly += dt * jy;
}

// The same step for an exact-reprojection flow: the chain to rho and theta
// per tap goes through the projection, translation and rotation of the set's
// pose (chain_exact).
__device__ __forceinline__ void adjoint_step(const WinParams& P, const FlowSrcX& u,
                                             const MotionXJ& mj, double X, double Y, double dt,
                                             double& Lx, double& Ly, double gl,
                                             float* __restrict__ drho, double (&dth)[6])
{
    const Taps tp = make_taps(P, X, Y);
    double2 uq[4];
    tap_flows(P, u, tp, uq);
    double jx = 0.0, jy = 0.0;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        double dX, dY;
        tap_dw(tp, q, dX, dY);
        const double lu = Lx * uq[q].x + Ly * uq[q].y;
        jx += lu * dX;
        jy += lu * dY;
        if (!tap_in(tp, q)) continue;
        const double w = tap_w(tp, q);
        if (w != 0.0) {
            const int i = tp.x0 + (q & 1), j = tp.y0 + (q >> 1);
            const int pix = j * P.W + i;
            const double gx = dt * w * Lx, gy = dt * w * Ly;
            const double d = chain_exact(P, mj, i, j, (double)u.rho[pix], gx, gy, dth);
            unsafeAtomicAdd(drho + pix, (float)(gl * d));
        }
    }
    Lx += dt * jx;
    Ly += dt * jy;
}

template <int RM, int FM>
__global__ __launch_bounds__(256) void backward_kernel(
    WinParams P, const float* __restrict__ ex, const float* __restrict__ ey,
    const float* __restrict__ et, const int8_t* __restrict__ ep, int64_t n,
    const float* __restrict__ rho, const float* __restrict__ ego,
    const double* __restrict__ img, const StateHeader* __restrict__ hdr,
    const float* __restrict__ grad_loss, float* __restrict__ drho, double* __restrict__ part)
{
    __shared__ double lds[16];
    __shared__ RefTable rt;
    __shared__ MotionTable mt;
    __shared__ MotionXJ mxj[FM == 2 ? kMaxFlows : 1];   // poses with right Jacobians (exact)
    if (threadIdx.x < kMaxRefs) {
        rt.t[threadIdx.x] = P.refs[threadIdx.x];
        rt.coef[threadIdx.x] =
            (int)threadIdx.x < P.R ? P.two_over_R / (hdr->nact[threadIdx.x] + P.eps) : 0.0;
        rt.sf[threadIdx.x] = P.sf[threadIdx.x];
        rt.sb[threadIdx.x] = P.sb[threadIdx.x];
    }
    if (FM == 2 && (int)threadIdx.x < P.F) mxj[threadIdx.x] = load_motion_xj(ego + 6 * threadIdx.x);
    const Flows<FM> u = make_flows<FM>(P, rho, ego, &mt);
    __syncthreads();
    const double gl = (double)grad_loss[0];
    // d theta partials: in registers with one flow set, per set in LDS with several
    __shared__ double dth_sets[FM ? kMaxFlows * 6 : 1];
    if (FM)
        for (int i = threadIdx.x; i < kMaxFlows * 6; i += blockDim.x) dth_sets[i] = 0.0;
    double dth[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};

    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n;
         k += (int64_t)gridDim.x * blockDim.x) {
        const double x0 = ex[k], y0 = ey[k], tk = et[k];
        const int pol = ep[k] > 0 ? 0 : 1;
        double vx[RM], vy[RM];
        Visits v;
        if (!warp_visits_v<RM, FM>(P, u, rt, x0, y0, tk, v, [&](int j, double X, double Y, int) {
                vx[j] = X;
                vy[j] = Y;
            }))
            continue;
        const double2* planes = reinterpret_cast<const double2*>(img) + (size_t)pol * P.HW;
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
                    const double X = s.first ? x0 : vx[j > 0 ? j - 1 : 0];
                    const double Y = s.first ? y0 : vy[j > 0 ? j - 1 : 0];
                    if (FM) {
                        double d6[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
                        if constexpr (FM == 2)
                            adjoint_step(P, u.at(s.set), mxj[s.set], X, Y, s.dt, Lx, Ly, gl,
                                         drho + (size_t)s.set * P.HW, d6);
                        else
                            adjoint_step(P, u.at(s.set), X, Y, s.dt, Lx, Ly, gl,
                                         drho + (size_t)s.set * P.HW, d6);
#pragma unroll
                        for (int c = 0; c < 6; ++c) atomicAdd(&dth_sets[s.set * 6 + c], d6[c]);
                    } else {
                        if constexpr (FM == 0) adjoint_step(P, u.at(0), X, Y, s.dt, Lx, Ly, gl, drho, dth);
                    }
                }
            }
        }
    }
    // part[block][set][6]
    if (FM) {
        __syncthreads();
        for (int i = threadIdx.x; i < P.F * 6; i += blockDim.x)
            part[(size_t)blockIdx.x * P.F * 6 + i] = dth_sets[i];
    } else {
#pragma unroll
        for (int c = 0; c < 6; ++c) {
            const double v = block_sum(dth[c], lds);
            if (threadIdx.x == 0) part[(size_t)blockIdx.x * 6 + c] = v;
        }
    }
}

__global__ __launch_bounds__(256) void finalize_backward_kernel(const double* __restrict__ part,
                                                                int nblk, int F,
                                                                const float* __restrict__ grad_loss,
                                                                float* __restrict__ grad_ego)
{
    __shared__ double lds[16];
    const double gl = (double)grad_loss[0];
    for (int f = 0; f < F; ++f)
        for (int c = 0; c < 6; ++c) {
            double s = 0.0;
            for (int b = threadIdx.x; b < nblk; b += blockDim.x)
                s += part[((size_t)b * F + f) * 6 + c];
            s = block_sum(s, lds);
            if (threadIdx.x == 0) grad_ego[f * 6 + c] = (float)(gl * s);
        }
}

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------

static int ceil_div(int64_t a, int64_t b) { return (int)((a + b - 1) / b); }

hipError_t launch_fill_zero(float* p, size_t n_floats, hipStream_t s)
{
    if (n_floats == 0) return hipSuccess;
    const int vec4 = (reinterpret_cast<uintptr_t>(p) % 16) == 0;
    const size_t work = vec4 ? n_floats / 4 + 1 : n_floats;
    const int grid = (int)std::min<size_t>((work + 255) / 256, 4096);
    fill_zero_kernel<<<std::max(grid, 1), 256, 0, s>>>(p, n_floats, vec4);
    return hipGetLastError();
}

template <int RM>
static void launch_splat_rm(const WinParams& P, const EventPtrs& ev, const float* rho,
                            const float* ego, double* img, unsigned long long* nv, hipStream_t s)
{
    const int grid = std::max(1, std::min(ceil_div(ev.n, 256), 1 << 20));
    if (P.model == 1)
        splat_kernel<RM, 2><<<grid, 256, 0, s>>>(P, ev.x, ev.y, ev.t, ev.p, ev.n, rho, ego, img, nv);
    else if (P.F > 1)
        splat_kernel<RM, 1><<<grid, 256, 0, s>>>(P, ev.x, ev.y, ev.t, ev.p, ev.n, rho, ego, img, nv);
    else
        splat_kernel<RM, 0><<<grid, 256, 0, s>>>(P, ev.x, ev.y, ev.t, ev.p, ev.n, rho, ego, img, nv);
}

template <int RM>
static void launch_backward_rm(const WinParams& P, const EventPtrs& ev, const float* rho,
                               const float* ego, const double* img, const StateHeader* hdr,
                               const float* gl, float* drho, double* part, int grid, hipStream_t s)
{
    if (P.model == 1)
        backward_kernel<RM, 2><<<grid, 256, 0, s>>>(P, ev.x, ev.y, ev.t, ev.p, ev.n, rho, ego,
                                                    img, hdr, gl, drho, part);
    else if (P.F > 1)
        backward_kernel<RM, 1><<<grid, 256, 0, s>>>(P, ev.x, ev.y, ev.t, ev.p, ev.n, rho, ego,
                                                    img, hdr, gl, drho, part);
    else
        backward_kernel<RM, 0><<<grid, 256, 0, s>>>(P, ev.x, ev.y, ev.t, ev.p, ev.n, rho, ego,
                                                    img, hdr, gl, drho, part);
}

int reduce_blocks(const WinParams& P) { return std::max(1, std::min(ceil_div(P.HW, 1024), kReduceBlocks)); }

int backward_blocks(int64_t n) { return std::max(1, std::min(ceil_div(n, 256), kBackwardBlocks)); }

hipError_t launch_forward(const WinParams& P, const EventPtrs& ev, const float* rho,
                          const float* ego, float* loss, const StatePtrs& st, hipStream_t s,
                          Profiler* prof)
{
    hipError_t e;
    {
        PhaseScope ph(prof, kPhZero, s);
        e = launch_fill_zero(reinterpret_cast<float*>(st.img), st.zero_floats, s);
    }
    if (e != hipSuccess) return e;
    if (ev.n > 0) {
        PhaseScope ph(prof, kPhSplat, s);
        if (P.R <= 2) launch_splat_rm<2>(P, ev, rho, ego, st.img, &st.hdr->n_valid, s);
        else if (P.R <= 4) launch_splat_rm<4>(P, ev, rho, ego, st.img, &st.hdr->n_valid, s);
        else if (P.R <= 8) launch_splat_rm<8>(P, ev, rho, ego, st.img, &st.hdr->n_valid, s);
        else launch_splat_rm<16>(P, ev, rho, ego, st.img, &st.hdr->n_valid, s);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    const int RB = reduce_blocks(P);
    {
        PhaseScope ph(prof, kPhReduce, s);
        reduce_kernel<<<dim3(RB, P.R), 256, 0, s>>>(P, st.img, st.scratch, RB);
        e = hipGetLastError();
    }
    if (e != hipSuccess) return e;
    {
        PhaseScope ph(prof, kPhFinalize, s);
        finalize_forward_kernel<<<1, 256, 0, s>>>(P, st.scratch, RB, st.hdr, loss);
        e = hipGetLastError();
    }
    return e;
}

hipError_t launch_backward(const WinParams& P, const EventPtrs& ev, const float* rho,
                           const float* ego, const StatePtrs& st, const float* grad_loss,
                           float* grad_rho, float* grad_ego, hipStream_t s, Profiler* prof)
{
    hipError_t e;
    {
        PhaseScope ph(prof, kPhGradZero, s);
        e = launch_fill_zero(grad_rho, (size_t)P.HW * P.F, s);
    }
    if (e != hipSuccess) return e;
    const int grid = backward_blocks(ev.n);
    if (ev.n > 0) {
        PhaseScope ph(prof, kPhAdjoint, s);
        if (P.R <= 2) launch_backward_rm<2>(P, ev, rho, ego, st.img, st.hdr, grad_loss, grad_rho, st.scratch, grid, s);
        else if (P.R <= 4) launch_backward_rm<4>(P, ev, rho, ego, st.img, st.hdr, grad_loss, grad_rho, st.scratch, grid, s);
        else if (P.R <= 8) launch_backward_rm<8>(P, ev, rho, ego, st.img, st.hdr, grad_loss, grad_rho, st.scratch, grid, s);
        else launch_backward_rm<16>(P, ev, rho, ego, st.img, st.hdr, grad_loss, grad_rho, st.scratch, grid, s);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    {
        PhaseScope ph(prof, kPhGradFinalize, s);
        finalize_backward_kernel<<<1, 256, 0, s>>>(st.scratch, ev.n > 0 ? grid : 0, P.F,
                                                   grad_loss, grad_ego);
        e = hipGetLastError();
    }
    return e;
}

}  // namespace cm
