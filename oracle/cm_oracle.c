/*
 * cm_oracle.c -- plain, slow FP64 CPU oracle for the contrast-maximization (CM)
 * loss and its gradient with respect to per-pixel inverse depth and ego-motion.
 *
 * TEST INFRASTRUCTURE.  Only the tests, the smoke check and the benchmark's
 * CPU-baseline leg may load this library.  It shares no code, header or
 * constant with the GPU library; the two meet only at the seeded inputs.
 *
 * What it computes (paper: Sec. 3.1 "Optical flow from contrast maximization",
 * Eq. 1; Sec. 3.2 "Combining depth and ego-motion into flow", Eq. 2; Fig. 2;
 * Sec. 3.3 on the per-event forward and the analytic backward):
 *
 *   1. A dense flow field u[H][W] from inverse depth rho and ego-motion
 *      theta = (v, w) through the first-order (motion-field) form of Eq. 2.
 *   2. Every event is pushed iteratively through the reference times, forward
 *      for the references after its timestamp and backward for those before,
 *      re-sampling the flow bilinearly at its current position at every step
 *      (the flow concatenation of Sec. 3.1).  An event that leaves the image at
 *      any visited reference time is masked for all of them.
 *   3. Surviving events are bilinearly splatted, per polarity and per reference
 *      time, into an image of warped events C and a timestamp-weighted image S.
 *   4. Eq. 1, read as the multi-reference average-timestamp loss:
 *        L = (1/R) sum_r [ sum_x sum_p (S_p/(C_p+eps))^2 ] / (N_r + eps),
 *      N_r = number of pixels with C_+ + C_- > 0 at reference r.
 *   5. The gradient: dL/du at every pixel (the quantity the paper's backward
 *      kernel produces), then chained through Eq. 2 to rho and theta.
 *
 * Flow sets (Sec. 3.1: flows of consecutive slices are concatenated,
 * Delta x_k = sum_i (Delta t_i u_i)(e_k)): the window holds either one flow,
 * or one flow per segment between consecutive knots {0, 1} U refs, each from
 * its own inverse depth and ego-motion.  A warp step moves between two
 * consecutive visited times, which always lie in one segment, and samples
 * that segment's flow.
 *
 * Readings of points the paper leaves open (each also listed in the design
 * notes): timestamp contribution tbar = 1 - |t_ref - t_k|; eps in both the
 * per-pixel ratio and the active-pixel normaliser; pixel centres at integer
 * coordinates and the image domain is the closed box [0,W-1] x [0,H-1];
 * bilinear taps outside the sensor are skipped (zero flow, zero splat);
 * flow units are pixels per unit of normalised window time; derivative of the
 * bilinear weights taken with the floor-based formula (right derivative at
 * integer positions).
 *
 * Everything is FP64: the arrays are taken in FP64 (FP32 data is widened
 * exactly by the caller).  No blocking, fusion or reordering beyond the steps
 * above.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define CMO_MAX_REFS 16

enum { CMO_OK = 0, CMO_BAD_ARG = -1, CMO_NO_MEM = -2 };

typedef struct {
    int W, H;
    double fx, fy, cx, cy;
    int R;
    double refs[CMO_MAX_REFS];
    double eps;
    int model;                      /* flow model: 0 first order, 1 exact reprojection */
    int F;                          /* flow sets: 1, or one per segment */
    int nk;                         /* knots: sorted unique {0, 1} U refs */
    double knots[CMO_MAX_REFS + 2];
    int kidx[CMO_MAX_REFS];         /* knot index of each reference */
} cmo_cam;

static int cmo_setup(cmo_cam* c, int W, int H, const double* K, int R, const double* refs,
                     double eps, int F, int model)
{
    if (model != 0 && model != 1) return CMO_BAD_ARG;
    c->model = model;
    if (W <= 0 || H <= 0 || !K || !refs || R < 1 || R > CMO_MAX_REFS) return CMO_BAD_ARG;
    c->W = W; c->H = H;
    c->fx = K[0]; c->fy = K[1]; c->cx = K[2]; c->cy = K[3];
    if (!(c->fx > 0.0) || !(c->fy > 0.0)) return CMO_BAD_ARG;
    c->R = R;
    for (int r = 0; r < R; ++r) {
        c->refs[r] = refs[r];
        if (!(c->refs[r] >= 0.0 && c->refs[r] <= 1.0)) return CMO_BAD_ARG;
        if (r > 0 && !(c->refs[r] > c->refs[r - 1])) return CMO_BAD_ARG;
    }
    c->eps = eps;
    /* knots: 0, the references, 1 (each once) */
    c->nk = 0;
    if (c->refs[0] > 0.0) c->knots[c->nk++] = 0.0;
    for (int r = 0; r < R; ++r) { c->kidx[r] = c->nk; c->knots[c->nk++] = c->refs[r]; }
    if (c->refs[R - 1] < 1.0) c->knots[c->nk++] = 1.0;
    if (F != 1 && F != c->nk - 1) return CMO_BAD_ARG;
    c->F = F;
    return CMO_OK;
}

/* Flow set of the step that ends at reference r: a forward step (from a
 * smaller time) crosses the segment that ends at r's knot, a backward step
 * the segment that starts there. */
static int cmo_set_fwd(const cmo_cam* c, int r) { return c->F == 1 ? 0 : c->kidx[r] - 1; }
static int cmo_set_bwd(const cmo_cam* c, int r) { return c->F == 1 ? 0 : c->kidx[r]; }

/* ---------------------------------------------------------------------------
 * Rotation by exponential coordinates (Rodrigues' formula, Sec. 3.2) and the
 * right Jacobian of the exponential map: R(w + d) = R(w) Exp(Jr(w) d) to
 * first order in d.  With theta = |w| and K = [w]x,
 *   R  = I + a K + b K^2,          a = sin(theta)/theta, b = (1 - cos theta)/theta^2
 *   Jr = I - b K + c K^2,          c = (theta - sin theta)/theta^3
 * (series in theta below 1e-4, where the closed forms lose digits).
 * ------------------------------------------------------------------------- */
static void cmo_skew(const double w[3], double K[9])
{
    K[0] = 0.0;   K[1] = -w[2]; K[2] = w[1];
    K[3] = w[2];  K[4] = 0.0;   K[5] = -w[0];
    K[6] = -w[1]; K[7] = w[0];  K[8] = 0.0;
}

static void cmo_matmul3(const double A[9], const double B[9], double C[9])
{
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            double acc = 0.0;
            for (int k = 0; k < 3; ++k) acc += A[3 * i + k] * B[3 * k + j];
            C[3 * i + j] = acc;
        }
}

static void cmo_rodrigues(const double w[3], double R[9], double Jr[9])
{
    const double t2 = w[0] * w[0] + w[1] * w[1] + w[2] * w[2];
    const double t = sqrt(t2);
    double a, b, c;
    if (t < 1e-4) {
        a = 1.0 - t2 / 6.0;
        b = 0.5 - t2 / 24.0;
        c = 1.0 / 6.0 - t2 / 120.0;
    } else {
        a = sin(t) / t;
        b = (1.0 - cos(t)) / t2;
        c = (t - sin(t)) / (t2 * t);
    }
    double K[9], K2[9];
    cmo_skew(w, K);
    cmo_matmul3(K, K, K2);
    for (int i = 0; i < 9; ++i) {
        const double I = (i % 4 == 0) ? 1.0 : 0.0;
        R[i] = I + a * K[i] + b * K2[i];
        Jr[i] = I - b * K[i] + c * K2[i];
    }
}

/* ---------------------------------------------------------------------------
 * Step 1b: flow from exact reprojection (Eq. 2 without the first-order
 * expansion).  A pixel's ray x0 = (xbar/fx, ybar/fy, 1) at inverse depth rho
 * is the point x0/rho; the pose maps it to R x0/rho + v, which projects like
 *   p = R x0 + rho v,   u = (fx p_x/p_z + cx - i, fy p_y/p_z + cy - j)
 * (depth cancels in the projection).  A point that lands on or behind the
 * camera plane (p_z <= 0) has no image: its flow is taken as zero, with zero
 * derivatives.
 * ------------------------------------------------------------------------- */
static int cmo_exact_point(const cmo_cam* c, int i, int j, double rho, const double th[6],
                           double p[3], double x0[3], double R[9], double Jr[9])
{
    cmo_rodrigues(th + 3, R, Jr);
    x0[0] = ((double)i - c->cx) / c->fx;
    x0[1] = ((double)j - c->cy) / c->fy;
    x0[2] = 1.0;
    for (int k = 0; k < 3; ++k)
        p[k] = R[3 * k + 0] * x0[0] + R[3 * k + 1] * x0[1] + R[3 * k + 2] * x0[2] + rho * th[k];
    return p[2] > 0.0;
}

static void cmo_flow_exact(const cmo_cam* c, int i, int j, double rho, const double th[6],
                           double u[2])
{
    double p[3], x0[3], R[9], Jr[9];
    if (!cmo_exact_point(c, i, j, rho, th, p, x0, R, Jr)) { u[0] = 0.0; u[1] = 0.0; return; }
    u[0] = c->fx * p[0] / p[2] + c->cx - (double)i;
    u[1] = c->fy * p[1] / p[2] + c->cy - (double)j;
}

/* ---------------------------------------------------------------------------
 * Step 1: flow from inverse depth and ego-motion (Eq. 2, first order).
 *
 * Back-project pixel x to X = D (xbar/fx, ybar/fy, 1), D = 1/rho, apply the
 * relative pose P = [R | t] with R ~ I + [w]x and t = v (P maps camera points
 * at window start to the frame at window end), re-project and keep the terms
 * of first order in (v, w):
 *   a1 = w_y - w_z ybar/fy + rho v_x
 *   a2 = w_z xbar/fx - w_x + rho v_y
 *   a3 = w_x ybar/fy - w_y xbar/fx + rho v_z
 *   u  = (fx a1 - xbar a3,  fy a2 - ybar a3)      [px per window]
 * with xbar = i - cx, ybar = j - cy.  Depth is defined up to scale (the "~" of
 * Eq. 2), so rho may be any positive multiple of 1/D with v scaled inversely.
 * ------------------------------------------------------------------------- */
static void cmo_flow_at(const cmo_cam* c, int i, int j, double rho, const double th[6],
                        double u[2])
{
    const double xb = (double)i - c->cx, yb = (double)j - c->cy;
    const double vx = th[0], vy = th[1], vz = th[2], wx = th[3], wy = th[4], wz = th[5];
    const double a1 = wy - wz * yb / c->fy + rho * vx;
    const double a2 = wz * xb / c->fx - wx + rho * vy;
    const double a3 = wx * yb / c->fy - wy * xb / c->fx + rho * vz;
    u[0] = c->fx * a1 - xb * a3;
    u[1] = c->fy * a2 - yb * a3;
}

static void cmo_fill_flow(const cmo_cam* c, const double* rho, const double* theta, double* u)
{
    double th[6];
    for (int k = 0; k < 6; ++k) th[k] = theta[k];
    for (int j = 0; j < c->H; ++j)
        for (int i = 0; i < c->W; ++i) {
            double* uij = &u[2 * ((size_t)j * c->W + i)];
            if (c->model == 1) cmo_flow_exact(c, i, j, rho[(size_t)j * c->W + i], th, uij);
            else cmo_flow_at(c, i, j, rho[(size_t)j * c->W + i], th, uij);
        }
}

/* ---------------------------------------------------------------------------
 * Bilinear kernel (the splatting kernel kappa of Eq. 1 and the "BS" sampling
 * of Fig. 2).  Taps in the order (x0,y0), (x0+1,y0), (x0,y0+1), (x0+1,y0+1)
 * with x0 = floor(X), a = X - x0 (same for y, b).
 * ------------------------------------------------------------------------- */
typedef struct {
    int xi[4], yi[4];
    int in[4];        /* tap lies on the sensor */
    double w[4];      /* weights */
    double dwx[4];    /* d w / d X (floor-based formula) */
    double dwy[4];    /* d w / d Y */
} cmo_taps;

static void cmo_bilinear(const cmo_cam* c, double X, double Y, cmo_taps* tp)
{
    const double x0 = floor(X), y0 = floor(Y);
    const double a = X - x0, b = Y - y0;
    const int ix = (int)x0, iy = (int)y0;
    const int ox[4] = {0, 1, 0, 1}, oy[4] = {0, 0, 1, 1};
    tp->w[0] = (1.0 - a) * (1.0 - b);
    tp->w[1] = a * (1.0 - b);
    tp->w[2] = (1.0 - a) * b;
    tp->w[3] = a * b;
    tp->dwx[0] = -(1.0 - b); tp->dwx[1] = (1.0 - b); tp->dwx[2] = -b;          tp->dwx[3] = b;
    tp->dwy[0] = -(1.0 - a); tp->dwy[1] = -a;        tp->dwy[2] = (1.0 - a);   tp->dwy[3] = a;
    for (int q = 0; q < 4; ++q) {
        tp->xi[q] = ix + ox[q];
        tp->yi[q] = iy + oy[q];
        tp->in[q] = tp->xi[q] >= 0 && tp->xi[q] < c->W && tp->yi[q] >= 0 && tp->yi[q] < c->H;
    }
}

static int cmo_inside(const cmo_cam* c, double X, double Y)
{
    return X >= 0.0 && X <= (double)(c->W - 1) && Y >= 0.0 && Y <= (double)(c->H - 1);
}

/* BS(u)(P): the flow sampled bilinearly at a real-valued position. */
static void cmo_sample(const cmo_cam* c, const double* u, double X, double Y, double out[2])
{
    cmo_taps tp;
    cmo_bilinear(c, X, Y, &tp);
    out[0] = 0.0; out[1] = 0.0;
    for (int q = 0; q < 4; ++q) {
        if (!tp.in[q]) continue;
        const double* uq = &u[2 * ((size_t)tp.yi[q] * c->W + tp.xi[q])];
        out[0] += tp.w[q] * uq[0];
        out[1] += tp.w[q] * uq[1];
    }
}

/* ---------------------------------------------------------------------------
 * Step 2: the iterative warp of one event (Sec. 3.1 flow concatenation;
 * Sec. 3.3 pushing each event forward or backward through time).
 *
 * From (x_k, t_k) the event is moved through the reference times after t_k in
 * increasing order, P <- P + (r - tau) BS(u_s)(P), tau <- r, with u_s the flow
 * of the segment the step crosses; then, from the original position again,
 * through the reference times before t_k in decreasing order.  A reference equal to t_k gets the unwarped position.
 * The event is valid iff its inputs are finite, t_k lies in [0,1], it starts
 * on the image and every visited position lies on the image.  pos[2r..2r+1]
 * receives the position at reference r.  Returns validity.
 * ------------------------------------------------------------------------- */
static int cmo_warp_event(const cmo_cam* c, const double* u, double xk, double yk, double tk,
                          double* pos)
{
    const size_t HW2 = 2 * (size_t)c->H * c->W;
    const int R = c->R;
    for (int r = 0; r < 2 * R; ++r) pos[r] = NAN;
    if (!isfinite(xk) || !isfinite(yk) || !isfinite(tk)) return 0;
    if (!(tk >= 0.0 && tk <= 1.0)) return 0;
    if (!cmo_inside(c, xk, yk)) return 0;

    int m = 0;                       /* number of refs strictly before t_k */
    while (m < R && c->refs[m] < tk) ++m;

    /* forward sweep */
    double X = xk, Y = yk, tau = tk;
    for (int r = m; r < R; ++r) {
        if (c->refs[r] == tk) { pos[2 * r] = xk; pos[2 * r + 1] = yk; continue; }
        double s[2];
        cmo_sample(c, u + HW2 * cmo_set_fwd(c, r), X, Y, s);
        const double dt = c->refs[r] - tau;
        X = X + dt * s[0];
        Y = Y + dt * s[1];
        tau = c->refs[r];
        if (!cmo_inside(c, X, Y)) return 0;
        pos[2 * r] = X; pos[2 * r + 1] = Y;
    }
    /* backward sweep */
    X = xk; Y = yk; tau = tk;
    for (int r = m - 1; r >= 0; --r) {
        double s[2];
        cmo_sample(c, u + HW2 * cmo_set_bwd(c, r), X, Y, s);
        const double dt = c->refs[r] - tau;
        X = X + dt * s[0];
        Y = Y + dt * s[1];
        tau = c->refs[r];
        if (!cmo_inside(c, X, Y)) return 0;
        pos[2 * r] = X; pos[2 * r + 1] = Y;
    }
    return 1;
}

/* Timestamp contribution of an event at t to the image at reference r. */
static double cmo_tbar(double r, double t) { return 1.0 - fabs(r - t); }

/* Image layout used by the oracle: img[((r*2 + pol)*2 + ch)*H*W + pix],
 * pol 0 = positive (p > 0), 1 = negative; ch 0 = C (warped-event count),
 * ch 1 = S (timestamp-weighted). */
static size_t cmo_img_index(const cmo_cam* c, int r, int pol, int ch, int xi, int yi)
{
    return (((size_t)r * 2 + pol) * 2 + ch) * (size_t)c->H * c->W + (size_t)yi * c->W + xi;
}

typedef struct {
    cmo_cam cam;
    double* u;      /* [F][H*W*2] flow */
    double* img;    /* [R*2*2*H*W] */
    double* nact;   /* [R] */
    double* num;    /* [R] */
    double loss;
} cmo_fwd;

static void cmo_fwd_free(cmo_fwd* f)
{
    free(f->u); free(f->img); free(f->nact); free(f->num);
}

/* Steps 1-4. */
static int cmo_forward_impl(cmo_fwd* f, int64_t n, const double* x, const double* y,
                            const double* t, const int8_t* p, const double* rho,
                            const double* theta, uint8_t* valid_out, double* pos_out)
{
    const cmo_cam* c = &f->cam;
    const int R = c->R;
    const size_t HW = (size_t)c->H * c->W;
    f->u = (double*)malloc(sizeof(double) * 2 * HW * (size_t)c->F);
    f->img = (double*)calloc((size_t)R * 4 * HW, sizeof(double));
    f->nact = (double*)calloc((size_t)R, sizeof(double));
    f->num = (double*)calloc((size_t)R, sizeof(double));
    if (!f->u || !f->img || !f->nact || !f->num) return CMO_NO_MEM;

    for (int fs = 0; fs < c->F; ++fs)
        cmo_fill_flow(c, rho + HW * fs, theta + 6 * fs, f->u + 2 * HW * fs);

    double pos[2 * CMO_MAX_REFS];
    for (int64_t k = 0; k < n; ++k) {
        const double tk = t[k];
        const int ok = cmo_warp_event(c, f->u, x[k], y[k], tk, pos);
        if (valid_out) valid_out[k] = (uint8_t)ok;
        if (pos_out) memcpy(&pos_out[(size_t)k * 2 * R], pos, sizeof(double) * 2 * R);
        if (!ok) continue;
        const int pol = p[k] > 0 ? 0 : 1;
        for (int r = 0; r < R; ++r) {
            cmo_taps tp;
            cmo_bilinear(c, pos[2 * r], pos[2 * r + 1], &tp);
            const double tb = cmo_tbar(c->refs[r], tk);
            for (int q = 0; q < 4; ++q) {
                if (!tp.in[q]) continue;
                f->img[cmo_img_index(c, r, pol, 0, tp.xi[q], tp.yi[q])] += tp.w[q];
                f->img[cmo_img_index(c, r, pol, 1, tp.xi[q], tp.yi[q])] += tp.w[q] * tb;
            }
        }
    }

    /* Eq. 1 with the active-pixel normalisation. */
    double total = 0.0;
    for (int r = 0; r < R; ++r) {
        double num = 0.0, nact = 0.0;
        for (int yi = 0; yi < c->H; ++yi)
            for (int xi = 0; xi < c->W; ++xi) {
                const double Cp = f->img[cmo_img_index(c, r, 0, 0, xi, yi)];
                const double Sp = f->img[cmo_img_index(c, r, 0, 1, xi, yi)];
                const double Cm = f->img[cmo_img_index(c, r, 1, 0, xi, yi)];
                const double Sm = f->img[cmo_img_index(c, r, 1, 1, xi, yi)];
                if (Cp + Cm > 0.0) nact += 1.0;
                const double Tp = Sp / (Cp + c->eps), Tm = Sm / (Cm + c->eps);
                num += Tp * Tp + Tm * Tm;
            }
        f->num[r] = num;
        f->nact[r] = nact;
        total += num / (nact + c->eps);
    }
    f->loss = total / (double)R;
    return CMO_OK;
}

/* ---------------------------------------------------------------------------
 * Public: flow field only (for tests of Eq. 2).
 * ------------------------------------------------------------------------- */
int cmo_flow_field(int W, int H, const double* K, const double* rho, const double* theta,
                   int model, double* u_out)
{
    cmo_cam c;
    const double one = 1.0;
    int st = cmo_setup(&c, W, H, K, 1, &one, 1e-9, 1, model);
    if (st) return st;
    if (!rho || !theta || !u_out) return CMO_BAD_ARG;
    cmo_fill_flow(&c, rho, theta, u_out);
    return CMO_OK;
}

/* ---------------------------------------------------------------------------
 * Public: forward.
 *   rho [F][H*W], theta [F][6] with F flow sets (1, or one per segment).
 *   out[0] = loss, out[1..R] = num_r, out[R+1..2R] = N_r.
 *   img (optional): [R][2 pol][2 (C,S)][H][W] FP64.
 *   valid (optional): [n] 0/1.   pos (optional): [n][R][2], NaN if unvisited.
 * ------------------------------------------------------------------------- */
int cmo_forward(int W, int H, const double* K, int R, const double* refs, double eps, int F,
                int model, int64_t n,
                const double* x, const double* y, const double* t, const int8_t* p,
                const double* rho, const double* theta, double* out, double* img,
                uint8_t* valid, double* pos)
{
    cmo_fwd f;
    memset(&f, 0, sizeof f);
    int st = cmo_setup(&f.cam, W, H, K, R, refs, eps, F, model);
    if (st) return st;
    if (n < 0 || !rho || !theta || !out || (n > 0 && (!x || !y || !t || !p)))
        return CMO_BAD_ARG;
    st = cmo_forward_impl(&f, n, x, y, t, p, rho, theta, valid, pos);
    if (st == CMO_OK) {
        out[0] = f.loss;
        for (int r = 0; r < R; ++r) { out[1 + r] = f.num[r]; out[1 + R + r] = f.nact[r]; }
        if (img) memcpy(img, f.img, sizeof(double) * (size_t)R * 4 * W * H);
    }
    cmo_fwd_free(&f);
    return st;
}

/* ---------------------------------------------------------------------------
 * Step 5: the gradient (Sec. 3.3: analytic partial derivatives with respect to
 * the flow, distributed bilinearly to the four nearest flow cells; then through
 * Eq. 2 to inverse depth and ego-motion).
 *
 * Seeds, with N_r and the event mask held fixed (both are piecewise constant):
 *   dL/dS_p(x,r) =  (2/R) S / ((C+eps)^2 (N_r+eps))
 *   dL/dC_p(x,r) = -(2/R) S^2 / ((C+eps)^3 (N_r+eps))
 * An event at position P on reference r adds w_q(P) to C and tbar w_q(P) to S
 * at its taps q, so its direct sensitivity is
 *   lambda(P) = sum_q (dL/dC + tbar dL/dS)(q) grad_P w_q(P).
 * Each warp step P_j = P_{j-1} + dt_j BS(u)(P_{j-1}) is then differentiated in
 * reverse order (adjoint Lam of the later position):
 *   dL/du(q of P_{j-1}) += dt_j w_q(P_{j-1}) Lam_j
 *   Lam_{j-1} = Lam_j + dt_j J(P_{j-1})^T Lam_j + lambda(P_{j-1}) [if a ref]
 * with J(P) = sum_q u_q (x) grad_P w_q(P); the adjoint of the fixed event
 * position is discarded.
 * ------------------------------------------------------------------------- */
static void cmo_direct(const cmo_cam* c, const double* img, const double* nact, int r, int pol,
                       double tb, double X, double Y, double lam[2])
{
    const double R = (double)c->R;
    cmo_taps tp;
    cmo_bilinear(c, X, Y, &tp);
    lam[0] = 0.0; lam[1] = 0.0;
    for (int q = 0; q < 4; ++q) {
        if (!tp.in[q]) continue;
        const double C = img[cmo_img_index(c, r, pol, 0, tp.xi[q], tp.yi[q])];
        const double S = img[cmo_img_index(c, r, pol, 1, tp.xi[q], tp.yi[q])];
        const double ce = C + c->eps, ne = nact[r] + c->eps;
        const double gS = (2.0 / R) * S / (ce * ce * ne);
        const double gC = -(2.0 / R) * S * S / (ce * ce * ce * ne);
        const double g = gC + tb * gS;
        lam[0] += g * tp.dwx[q];
        lam[1] += g * tp.dwy[q];
    }
}

/* Reverse pass over one sweep: path[0] is the event, path[1..len] the visited
 * reference positions with reference indices ridx[1..len] and times tau; the
 * step into path[j] used flow set fset[j] (u and dflow are [F][H*W*2]). */
static void cmo_reverse_sweep(const cmo_cam* c, const double* u, const double* img,
                              const double* nact, int pol, double tk, int len,
                              const double* px, const double* py, const double* tau,
                              const int* ridx, const int* fset, double* dflow_all)
{
    const size_t HW2 = 2 * (size_t)c->H * c->W;
    double Lx = 0.0, Ly = 0.0;
    for (int j = len; j >= 1; --j) {
        double lam[2];
        const int r = ridx[j];
        cmo_direct(c, img, nact, r, pol, cmo_tbar(c->refs[r], tk), px[j], py[j], lam);
        Lx += lam[0];
        Ly += lam[1];
        const double dt = tau[j] - tau[j - 1];
        const double* us = u + HW2 * fset[j];
        double* dflow = dflow_all + HW2 * fset[j];
        cmo_taps tp;
        cmo_bilinear(c, px[j - 1], py[j - 1], &tp);
        double jx = 0.0, jy = 0.0;   /* J(P_{j-1})^T Lam */
        for (int q = 0; q < 4; ++q) {
            if (!tp.in[q]) continue;
            const size_t pix = (size_t)tp.yi[q] * c->W + tp.xi[q];
            dflow[2 * pix] += dt * tp.w[q] * Lx;
            dflow[2 * pix + 1] += dt * tp.w[q] * Ly;
            const double lu = Lx * us[2 * pix] + Ly * us[2 * pix + 1];
            jx += lu * tp.dwx[q];
            jy += lu * tp.dwy[q];
        }
        Lx = Lx + dt * jx;
        Ly = Ly + dt * jy;
    }
}

/* Exact model: with J = du/dp = [[fx/pz, 0, -fx px/pz^2], [0, fy/pz, -fy py/pz^2]]
 * and q = J^T g,
 *   d rho  += q . v,     d v += rho q,     d w += (d(R x0)/dw)^T q,
 *   d(R x0)/dw = -R [x0]x Jr(w)   (so (.)^T q = -Jr^T [x0]x^T R^T q = Jr^T (x0 x (R^T q))). */
static void cmo_chain_exact_pixel(const cmo_cam* c, int i, int j, double rho,
                                  const double th[6], double gx, double gy, double* drho,
                                  double dth[6])
{
    double p[3], x0[3], R[9], Jr[9];
    *drho = 0.0;
    if (!cmo_exact_point(c, i, j, rho, th, p, x0, R, Jr)) return;
    const double iz = 1.0 / p[2];
    const double q[3] = {gx * c->fx * iz, gy * c->fy * iz,
                         -(gx * c->fx * p[0] + gy * c->fy * p[1]) * iz * iz};
    *drho = q[0] * th[0] + q[1] * th[1] + q[2] * th[2];
    for (int k = 0; k < 3; ++k) dth[k] += rho * q[k];
    double s[3];                                   /* R^T q */
    for (int k = 0; k < 3; ++k) s[k] = R[0 * 3 + k] * q[0] + R[1 * 3 + k] * q[1] + R[2 * 3 + k] * q[2];
    const double cr[3] = {x0[1] * s[2] - x0[2] * s[1], x0[2] * s[0] - x0[0] * s[2],
                          x0[0] * s[1] - x0[1] * s[0]};   /* x0 x (R^T q) */
    for (int k = 0; k < 3; ++k)
        dth[3 + k] += Jr[0 * 3 + k] * cr[0] + Jr[1 * 3 + k] * cr[1] + Jr[2 * 3 + k] * cr[2];
}

/* Chain dL/du through Eq. 2 (first order, or exact) to rho and theta. */
static void cmo_chain(const cmo_cam* c, const double* rho, const double* theta,
                      const double* dflow, double* drho, double* dth)
{
    const double vx = theta[0], vy = theta[1], vz = theta[2];
    for (int k = 0; k < 6; ++k) dth[k] = 0.0;
    for (int j = 0; j < c->H; ++j)
        for (int i = 0; i < c->W; ++i) {
            const size_t pix = (size_t)j * c->W + i;
            const double gx = dflow[2 * pix], gy = dflow[2 * pix + 1];
            if (c->model == 1) {
                cmo_chain_exact_pixel(c, i, j, rho[pix], theta, gx, gy, &drho[pix], dth);
                continue;
            }
            const double xb = (double)i - c->cx, yb = (double)j - c->cy;
            const double rh = rho[pix];
            /* u_x = fx a1 - xb a3, u_y = fy a2 - yb a3 */
            const double da1[6] = {rh, 0.0, 0.0, 0.0, 1.0, -yb / c->fy};
            const double da2[6] = {0.0, rh, 0.0, -1.0, 0.0, xb / c->fx};
            const double da3[6] = {0.0, 0.0, rh, yb / c->fy, -xb / c->fx, 0.0};
            for (int k = 0; k < 6; ++k)
                dth[k] += gx * (c->fx * da1[k] - xb * da3[k]) + gy * (c->fy * da2[k] - yb * da3[k]);
            drho[pix] = gx * (c->fx * vx - xb * vz) + gy * (c->fy * vy - yb * vz);
        }
}

/* ---------------------------------------------------------------------------
 * Public: backward.  Recomputes the forward, then, per flow set,
 *   drho [F][H*W] = grad_loss * dL/drho,  dtheta [F][6] = grad_loss * dL/dtheta,
 *   dflow (optional) [F][H*W*2] = grad_loss * dL/du.
 * ------------------------------------------------------------------------- */
int cmo_backward(int W, int H, const double* K, int R, const double* refs, double eps, int F,
                 int model, int64_t n,
                 const double* x, const double* y, const double* t, const int8_t* p,
                 const double* rho, const double* theta, double grad_loss, double* drho,
                 double* dtheta, double* dflow_out)
{
    cmo_fwd f;
    memset(&f, 0, sizeof f);
    int st = cmo_setup(&f.cam, W, H, K, R, refs, eps, F, model);
    if (st) return st;
    if (n < 0 || !rho || !theta || !drho || !dtheta || (n > 0 && (!x || !y || !t || !p)))
        return CMO_BAD_ARG;
    st = cmo_forward_impl(&f, n, x, y, t, p, rho, theta, NULL, NULL);
    if (st) { cmo_fwd_free(&f); return st; }
    const cmo_cam* c = &f.cam;
    const size_t HW = (size_t)H * W;
    double* dflow = (double*)calloc(2 * HW * (size_t)F, sizeof(double));
    if (!dflow) { cmo_fwd_free(&f); return CMO_NO_MEM; }

    double pos[2 * CMO_MAX_REFS];
    double px[CMO_MAX_REFS + 1], py[CMO_MAX_REFS + 1], tau[CMO_MAX_REFS + 1];
    int ridx[CMO_MAX_REFS + 1], fset[CMO_MAX_REFS + 1];
    for (int64_t k = 0; k < n; ++k) {
        const double tk = t[k];
        if (!cmo_warp_event(c, f.u, x[k], y[k], tk, pos)) continue;
        const int pol = p[k] > 0 ? 0 : 1;
        int m = 0;
        while (m < R && c->refs[m] < tk) ++m;
        /* forward sweep path: refs after t_k in increasing order */
        int len = 0;
        px[0] = x[k]; py[0] = y[k]; tau[0] = tk; ridx[0] = -1;
        for (int r = m; r < R; ++r) {
            if (c->refs[r] == tk) continue;
            ++len;
            px[len] = pos[2 * r]; py[len] = pos[2 * r + 1]; tau[len] = c->refs[r]; ridx[len] = r;
            fset[len] = cmo_set_fwd(c, r);
        }
        cmo_reverse_sweep(c, f.u, f.img, f.nact, pol, tk, len, px, py, tau, ridx, fset, dflow);
        /* backward sweep path: refs before t_k in decreasing order */
        len = 0;
        for (int r = m - 1; r >= 0; --r) {
            ++len;
            px[len] = pos[2 * r]; py[len] = pos[2 * r + 1]; tau[len] = c->refs[r]; ridx[len] = r;
            fset[len] = cmo_set_bwd(c, r);
        }
        cmo_reverse_sweep(c, f.u, f.img, f.nact, pol, tk, len, px, py, tau, ridx, fset, dflow);
    }
    for (size_t i = 0; i < 2 * HW * (size_t)F; ++i) dflow[i] *= grad_loss;
    for (int fs = 0; fs < F; ++fs)
        cmo_chain(c, rho + HW * fs, theta + 6 * fs, dflow + 2 * HW * fs, drho + HW * fs,
                  dtheta + 6 * fs);
    if (dflow_out) memcpy(dflow_out, dflow, sizeof(double) * 2 * HW * (size_t)F);
    free(dflow);
    cmo_fwd_free(&f);
    return CMO_OK;
}

/* ===========================================================================
 * Geometry consistency between consecutive flow sets (Sec. 3.2, Eq. 3) and
 * the full loss (Eq. 4: L = L_CM + lambda L_geo, lambda = 0.05 in the paper's
 * training set-up).
 *
 * The paper gives Eq. 3 and takes the rest from Bian et al.'s scale-consistency
 * loss.  Readings:
 *  - The depth of flow set f is D_f = 1/rho_f.  Consecutive sets f and f+1
 *    form a pair.  The relative pose from set f's camera to set f+1's is the
 *    motion over segment f at set f's velocity: rotation R = Exp(Delta_f w_f)
 *    (Rodrigues) and translation t = Delta_f v_f, with Delta_f = k_{f+1} - k_f
 *    the segment's length; a point maps as X -> R X + t, the convention of
 *    Eq. 2's flow.
 *  - Pixel x of set f back-projects to X = x0 / rho_f(x), x0 = ((i - cx)/fx,
 *    (j - cy)/fy, 1).  The forward-projected depth D_{0->1}(x) is the z of
 *    P = R X + t.  The interpolated depth D'_1(x) is the bilinear
 *    interpolation of D_{f+1} at P's projection x' = (fx Px/Pz + cx,
 *    fy Py/Pz + cy), over the taps that lie on the sensor.
 *  - V (visible in both images): rho_f(x) > 0, Pz > 0, x' in the closed box
 *    [0, W-1] x [0, H-1], and rho_{f+1} > 0 at every on-sensor tap of x'.
 *  - L_geo of a window = mean over its F-1 pairs of the pair's mean over V of
 *    |D_{0->1} - D'_1| / (D_{0->1} + D'_1).  An empty V gives that pair 0; a
 *    window with one flow set has no pair and L_geo = 0.
 *  - Derivative: |V| is held constant (it changes only where a pixel crosses
 *    the validity boundary), d|d|/dd = sign(d) with sign(0) = 0, bilinear
 *    weights differentiated with the floor-based formula.
 * ======================================================================== */

/* One pixel of a pair.  Returns 1 if x is in V; fills the scaled point
 * p = rho_a P = R x0 + rho_a t, the taps of x', a = D_{0->1} = p_z / rho_a and
 * b = D'_1.  x' is formed as the pixel plus its displacement,
 * x' = i + fx (p_x/p_z - x0_x) (algebraically fx p_x/p_z + cx), so that zero
 * motion maps every pixel exactly onto itself. */
static int cmo_geo_pixel(const cmo_cam* c, int i, int j, double rho_a, const double* rho_b,
                         const double R[9], const double t[3], double x0[3], double p[3],
                         cmo_taps* tp, double* a, double* b)
{
    if (!(rho_a > 0.0)) return 0;
    x0[0] = ((double)i - c->cx) / c->fx;
    x0[1] = ((double)j - c->cy) / c->fy;
    x0[2] = 1.0;
    for (int k = 0; k < 3; ++k)
        p[k] = R[3 * k + 0] * x0[0] + R[3 * k + 1] * x0[1] + R[3 * k + 2] * x0[2] + rho_a * t[k];
    if (!(p[2] > 0.0)) return 0;
    const double xs = (double)i + c->fx * (p[0] / p[2] - x0[0]);
    const double ys = (double)j + c->fy * (p[1] / p[2] - x0[1]);
    if (!cmo_inside(c, xs, ys)) return 0;
    cmo_bilinear(c, xs, ys, tp);
    *b = 0.0;
    for (int q = 0; q < 4; ++q) {
        if (!tp->in[q]) continue;
        const double rb = rho_b[(size_t)tp->yi[q] * c->W + tp->xi[q]];
        if (!(rb > 0.0)) return 0;
        *b += tp->w[q] / rb;
    }
    *a = p[2] / rho_a;
    return 1;
}

static void cmo_pair_pose(const cmo_cam* c, const double* theta, int f, double R[9],
                          double Jr[9], double t[3], double* delta)
{
    *delta = c->knots[f + 1] - c->knots[f];
    const double w[3] = {*delta * theta[6 * f + 3], *delta * theta[6 * f + 4],
                         *delta * theta[6 * f + 5]};
    cmo_rodrigues(w, R, Jr);
    for (int k = 0; k < 3; ++k) t[k] = *delta * theta[6 * f + k];
}

/* Public: L_geo of one window (F >= 1 flow sets, rho [F][H*W], theta [F][6]).
 * loss receives L_geo; pair_out (optional, [F-1][2]) the per-pair (mean over
 * V, |V|); drho [F][H*W] and dtheta [F][6] (optional, both or neither)
 * receive grad_loss * dL_geo/d(.). */
int cmo_geo(int W, int H, const double* K, int R, const double* refs, int F,
            const double* rho, const double* theta, double grad_loss, double* loss,
            double* pair_out, double* drho, double* dtheta)
{
    cmo_cam cam;
    int st = cmo_setup(&cam, W, H, K, R, refs, 1e-9, F, 0);
    if (st) return st;
    if (!rho || !theta || !loss || (!drho) != (!dtheta)) return CMO_BAD_ARG;
    const cmo_cam* c = &cam;
    const size_t HW = (size_t)H * W;
    *loss = 0.0;
    if (drho) {
        memset(drho, 0, sizeof(double) * HW * (size_t)F);
        memset(dtheta, 0, sizeof(double) * 6 * (size_t)F);
    }
    if (F < 2) return CMO_OK;
    for (int f = 0; f + 1 < F; ++f) {
        double Rm[9], Jr[9], t[3], delta;
        cmo_pair_pose(c, theta, f, Rm, Jr, t, &delta);
        const double* ra = rho + HW * f;
        const double* rb = rho + HW * (f + 1);
        double sum = 0.0, nv = 0.0;
        for (int j = 0; j < H; ++j)
            for (int i = 0; i < W; ++i) {
                double x0[3], pp[3], a, b;
                cmo_taps tp;
                if (!cmo_geo_pixel(c, i, j, ra[(size_t)j * W + i], rb, Rm, t, x0, pp, &tp, &a, &b))
                    continue;
                sum += fabs(a - b) / (a + b);
                nv += 1.0;
            }
        const double mean = nv > 0.0 ? sum / nv : 0.0;
        *loss += mean / (double)(F - 1);
        if (pair_out) { pair_out[2 * f] = mean; pair_out[2 * f + 1] = nv; }
        if (!drho || nv == 0.0) continue;
        /* backward of the pair */
        const double cf = grad_loss / ((double)(F - 1) * nv);
        double* dra = drho + HW * f;
        double* drb = drho + HW * (f + 1);
        double dpose[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
        for (int j = 0; j < H; ++j)
            for (int i = 0; i < W; ++i) {
                const double rho_a = ra[(size_t)j * W + i];
                double x0[3], pp[3], a, b;
                cmo_taps tp;
                if (!cmo_geo_pixel(c, i, j, rho_a, rb, Rm, t, x0, pp, &tp, &a, &b)) continue;
                const double s = a > b ? 1.0 : (a < b ? -1.0 : 0.0);
                const double den = (a + b) * (a + b);
                const double ga = cf * s * 2.0 * b / den;      /* d/da of |a-b|/(a+b) */
                const double gb = -cf * s * 2.0 * a / den;     /* d/db */
                /* b = sum_q w_q / rho_b[q] */
                double dbx = 0.0, dby = 0.0;
                for (int q = 0; q < 4; ++q) {
                    if (!tp.in[q]) continue;
                    const size_t pq = (size_t)tp.yi[q] * W + tp.xi[q];
                    drb[pq] += gb * tp.w[q] * (-1.0 / (rb[pq] * rb[pq]));
                    dbx += tp.dwx[q] / rb[pq];
                    dby += tp.dwy[q] / rb[pq];
                }
                /* x' = i + fx (p_x/p_z - x0_x), y' likewise, a = p_z / rho_a */
                const double gxs = gb * dbx, gys = gb * dby;
                const double gp[3] = {gxs * c->fx / pp[2], gys * c->fy / pp[2],
                                      ga / rho_a - (gxs * c->fx * pp[0] + gys * c->fy * pp[1]) / (pp[2] * pp[2])};
                /* p = R x0 + rho_a t */
                dra[(size_t)j * W + i] += gp[0] * t[0] + gp[1] * t[1] + gp[2] * t[2]
                                          - ga * pp[2] / (rho_a * rho_a);
                for (int k = 0; k < 3; ++k) dpose[k] += rho_a * gp[k];
                /* d(R x0)/dw = -R [x0]x Jr  =>  dw += Jr^T (x0 x (R^T gp)) */
                double sv[3];
                for (int k = 0; k < 3; ++k)
                    sv[k] = Rm[0 * 3 + k] * gp[0] + Rm[1 * 3 + k] * gp[1] + Rm[2 * 3 + k] * gp[2];
                const double cr[3] = {x0[1] * sv[2] - x0[2] * sv[1], x0[2] * sv[0] - x0[0] * sv[2],
                                      x0[0] * sv[1] - x0[1] * sv[0]};
                for (int k = 0; k < 3; ++k)
                    dpose[3 + k] += Jr[0 * 3 + k] * cr[0] + Jr[1 * 3 + k] * cr[1] + Jr[2 * 3 + k] * cr[2];
            }
        /* pose = Delta_f theta_f */
        for (int k = 0; k < 6; ++k) dtheta[6 * f + k] += delta * dpose[k];
    }
    return CMO_OK;
}
