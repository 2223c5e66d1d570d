/*
 * cm_mirror.c -- CPU replica of the deterministic mode's canonical operation
 * order, for bit-exact comparison with the GPU.
 *
 * TEST INFRASTRUCTURE.  This is not the oracle: the FP64 oracle (cm_oracle.c)
 * states what the loss is; this file states in which order the deterministic
 * mode adds things up, and follows that order operation by operation so that
 * its results are bit-identical to a correct deterministic implementation.  It
 * shares no code with the GPU library.
 *
 * The canonical order (the contract of the deterministic mode):
 *  - Per-window constants: fx, fy, cx, cy, refs, eps widened from FP32;
 *    inv_fx = 1/fx, inv_fy = 1/fy, fx/fy, fy/fx, 2/R in FP64.
 *  - Motion coefficients k0 = fx w_y, k1 = (fx/fy) w_z, k2 = w_x inv_fy,
 *    k3 = w_y inv_fx, k4 = -(fy w_x), k5 = (fy/fx) w_z, tvx = fx v_x,
 *    tvy = fy v_y; the flow at pixel (i, j) with xb = i - cx, yb = j - cy:
 *    s = k3 xb - k2 yb, Ax = (k0 - k1 yb) + xb s, Ay = (k4 + k5 xb) + yb s,
 *    Bx = tvx - xb vz, By = tvy - yb vz, u = (Ax + rho Bx, Ay + rho By).
 *    Every operation is a separate IEEE FP64 operation (no fused multiply-add).
 *  - Exact flow (Eq. 2 without the first-order expansion): with t^2 = s =
 *    (wx^2 + wy^2) + wz^2 and series(s, o) = 1 - (s/d_1)(1 - (s/d_2)(...)),
 *    d_k = (o + 2k - 1)(o + 2k), 18 terms, Horner from the innermost:
 *    a = series(s, 1), b = 0.5 series(s, 2), c = series(s, 3) / 6;
 *    K = [w]x, K2 = K K (entries (K_i0 K_0j + K_i1 K_1j) + K_i2 K_2j),
 *    R = (I + a K) + b K2, Jr = (I - b K) + c K2.  At pixel (i, j):
 *    xn = (i - cx) inv_fx, yn = (j - cy) inv_fy,
 *    p_k = (R_k0 xn + (R_k1 yn + R_k2)) + rho v_k; if p_z > 0, iz = 1/p_z,
 *    u = ((fx p_x) iz + (cx - i), (fy p_y) iz + (cy - j)), else u = 0.
 *    The chain of dL/du = g at a pixel: ax = gx fx, ay = gy fy,
 *    q = (ax iz, ay iz, -((ax p_x + ay p_y) iz) iz), d rho = (q_x v_x + q_y v_y)
 *    + q_z v_z, d v_k += rho q_k, s_k = (R_0k q_x + R_1k q_y) + R_2k q_z,
 *    c = (yn s_z - s_y, s_x - xn s_z, xn s_y - yn s_x),
 *    d w_k += (Jr_0k c_0 + Jr_1k c_1) + Jr_2k c_2.
 *  - Bilinear sample: ux = ((((0 + w0 u0) + w1 u1) + w2 u2) + w3 u3) with
 *    u = 0 for taps off the sensor; w_q = wa * wb.
 *  - Warp: one loop over the visits (forward references from t_k upward, then
 *    backward references downward), P += (ref - tau) * u.
 *  - Events are grouped in blocks of 64 * ept consecutive events, ept =
 *    clamp(n / 65536, 1, 16); records of a bin are ordered by (block,
 *    iteration e, program point, lane); in the forward that is event order.
 *    The backward's blocks run over the valid events in source order (grouped
 *    by the tile of their reference-0 position, event order within a tile),
 *    interleaved: iteration e of block b takes positions (e nblocks + b) 64 ..;
 *    its program points are the visits j = R-1 .. 0 (visits: the forward
 *    sweep's references at or after t_k upward, then the backward sweep's
 *    downward), then the event's own record.
 *  - Tile accumulation: records of a (reference, 32x32 tile) bin, 64 at a
 *    time; for tap slot q = 0..3, then lane 0..63, the record's (w, w tbar) is
 *    added to its cell.  Halos (right column rows 0..32, bottom row) are added
 *    to the neighbours' column 0 / row 0 in the order left, top, top-left.
 *  - Reductions: per thread in index order, then a 64-lane shuffle-down tree
 *    (offsets 32..1), then the per-wavefront results in order.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define MM_MAX_REFS 16
#define TW 32
#define TH 32
#define TLW 33
#define TLH 33
#define NHALO (TH + 1 + TW)
#define NBORDER (TW + TH - 1)

enum { MM_OK = 0, MM_BAD = -1, MM_NOMEM = -2 };

#define MM_MAX_FLOWS (MM_MAX_REFS + 1)

typedef struct {
    int W, H, R, HW;
    double cx, cy, fx, fy, inv_fx, inv_fy, fx_over_fy, fy_over_fx, xmax, ymax, eps, two_over_R;
    double refs[MM_MAX_REFS];
    /* flow sets: motion per set, inverse depth of set f at rho + f HW; the step
     * into reference r uses set sf[r] forward in time, sb[r] backward */
    int F;
    double k0[MM_MAX_FLOWS], k1[MM_MAX_FLOWS], k2[MM_MAX_FLOWS], k3[MM_MAX_FLOWS];
    double k4[MM_MAX_FLOWS], k5[MM_MAX_FLOWS], tvx[MM_MAX_FLOWS], tvy[MM_MAX_FLOWS];
    double vz[MM_MAX_FLOWS];
    int sf[MM_MAX_REFS], sb[MM_MAX_REFS];
    /* exact flow (model 1): rotation, translation, right Jacobian per set */
    int model;
    double Rm[MM_MAX_FLOWS][9], v[MM_MAX_FLOWS][3], Jr[MM_MAX_FLOWS][9];
    const float* rho;
    /* tiles */
    int ntx, nty, ntiles, ept, nblocks;
} mm_win;

typedef struct { double x, y; } d2;

static double mm_series(double s, int o)
{
    double h = 1.0;
    for (int k = 18; k >= 1; --k) {
        const double d = (double)(o + 2 * k - 1) * (double)(o + 2 * k);
        h = 1.0 - (s / d) * h;
    }
    return h;
}

static void mm_rotation(const float* th, double* Rm, double* Jr)
{
    const double wx = th[3], wy = th[4], wz = th[5];
    const double s = (wx * wx + wy * wy) + wz * wz;
    const double a = mm_series(s, 1), b = 0.5 * mm_series(s, 2), c = mm_series(s, 3) / 6.0;
    const double K[9] = {0.0, -wz, wy, wz, 0.0, -wx, -wy, wx, 0.0};
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            const double k2 = (K[3 * i] * K[j] + K[3 * i + 1] * K[3 + j]) + K[3 * i + 2] * K[6 + j];
            const double I = i == j ? 1.0 : 0.0;
            Rm[3 * i + j] = (I + a * K[3 * i + j]) + b * k2;
            Jr[3 * i + j] = (I - b * K[3 * i + j]) + c * k2;
        }
}

static int mm_setup(mm_win* w, int W, int H, const float* K, int R, const float* refs, float eps,
                    int F, int model, const float* rho, const float* theta, int64_t n)
{
    if (W <= 0 || H <= 0 || R < 1 || R > MM_MAX_REFS || (model != 0 && model != 1)) return MM_BAD;
    memset(w, 0, sizeof *w);
    w->W = W; w->H = H; w->R = R; w->HW = W * H;
    w->fx = K[0]; w->fy = K[1]; w->cx = K[2]; w->cy = K[3];
    w->inv_fx = 1.0 / w->fx; w->inv_fy = 1.0 / w->fy;
    w->fx_over_fy = w->fx / w->fy; w->fy_over_fx = w->fy / w->fx;
    w->xmax = (double)(W - 1); w->ymax = (double)(H - 1);
    w->eps = eps;
    w->two_over_R = 2.0 / (double)R;
    for (int r = 0; r < R; ++r) w->refs[r] = refs[r];
    /* knots {0, 1} U refs; segment f between knots f and f+1 */
    const int k0 = refs[0] > 0.f ? 1 : 0;
    const int nseg = R - 1 + k0 + (refs[R - 1] < 1.f ? 1 : 0);
    if (F != 1 && F != nseg) return MM_BAD;
    w->F = F;
    for (int r = 0; r < R; ++r) {
        w->sf[r] = F > 1 ? (k0 + r - 1 > 0 ? k0 + r - 1 : 0) : 0;
        w->sb[r] = F > 1 ? (k0 + r < F - 1 ? k0 + r : F - 1) : 0;
    }
    for (int f = 0; f < F; ++f) {
        const float* th = theta + 6 * f;
        const double vx = th[0], vy = th[1], vz = th[2];
        const double wx = th[3], wy = th[4], wz = th[5];
        w->k0[f] = w->fx * wy;
        w->k1[f] = w->fx_over_fy * wz;
        w->k2[f] = wx * w->inv_fy;
        w->k3[f] = wy * w->inv_fx;
        w->k4[f] = -w->fy * wx;
        w->k5[f] = w->fy_over_fx * wz;
        w->tvx[f] = w->fx * vx;
        w->tvy[f] = w->fy * vy;
        w->vz[f] = vz;
        mm_rotation(th, w->Rm[f], w->Jr[f]);
        w->v[f][0] = vx; w->v[f][1] = vy; w->v[f][2] = vz;
    }
    w->model = model;
    w->rho = rho;
    w->ntx = (W + TW - 1) / TW;
    w->nty = (H + TH - 1) / TH;
    w->ntiles = w->ntx * w->nty;
    int64_t ept = n / (64 * 1024);
    if (ept < 1) ept = 1;
    if (ept > 16) ept = 16;
    w->ept = (int)ept;
    const int64_t per = 64 * ept;
    w->nblocks = (int)((n + per - 1) / per);
    if (w->nblocks < 1) w->nblocks = 1;
    return MM_OK;
}

static void mm_parts(const mm_win* w, int f, int i, int j, double* Ax, double* Ay, double* Bx,
                     double* By)
{
    const double xb = (double)i - w->cx;
    const double yb = (double)j - w->cy;
    const double s = w->k3[f] * xb - w->k2[f] * yb;
    *Ax = (w->k0[f] - w->k1[f] * yb) + xb * s;
    *Ay = (w->k4[f] + w->k5[f] * xb) + yb * s;
    *Bx = w->tvx[f] - xb * w->vz[f];
    *By = w->tvy[f] - yb * w->vz[f];
}

/* the exact model's camera-frame point of pixel (i, j) after the motion */
static void mm_point(const mm_win* w, int f, int i, int j, double r, double* xn, double* yn,
                     double p[3])
{
    const double* Rm = w->Rm[f];
    *xn = ((double)i - w->cx) * w->inv_fx;
    *yn = ((double)j - w->cy) * w->inv_fy;
    for (int k = 0; k < 3; ++k)
        p[k] = (Rm[3 * k] * *xn + (Rm[3 * k + 1] * *yn + Rm[3 * k + 2])) + r * w->v[f][k];
}

static d2 mm_flow(const mm_win* w, int f, int i, int j)
{
    if (w->model == 1) {
        const double r = (double)w->rho[(size_t)f * w->HW + j * w->W + i];
        double xn, yn, p[3];
        mm_point(w, f, i, j, r, &xn, &yn, p);
        d2 u = {0.0, 0.0};
        if (p[2] > 0.0) {
            const double iz = 1.0 / p[2];
            u.x = (w->fx * p[0]) * iz + (w->cx - (double)i);
            u.y = (w->fy * p[1]) * iz + (w->cy - (double)j);
        }
        return u;
    }
    double Ax, Ay, Bx, By;
    mm_parts(w, f, i, j, &Ax, &Ay, &Bx, &By);
    const double r = (double)w->rho[(size_t)f * w->HW + j * w->W + i];
    d2 u = {Ax + r * Bx, Ay + r * By};
    return u;
}

typedef struct { int x0, y0; double a, b; int inx, iny; } mm_taps;

static mm_taps mm_make_taps(const mm_win* w, double X, double Y)
{
    mm_taps t;
    const double fx0 = floor(X), fy0 = floor(Y);
    t.x0 = (int)fx0; t.y0 = (int)fy0;
    t.a = X - fx0; t.b = Y - fy0;
    t.inx = t.x0 + 1 < w->W;
    t.iny = t.y0 + 1 < w->H;
    return t;
}

static int mm_tap_in(const mm_taps* t, int q) { return ((q & 1) ? t->inx : 1) && ((q & 2) ? t->iny : 1); }

static double mm_tap_w(const mm_taps* t, int q)
{
    const double wa = (q & 1) ? t->a : 1.0 - t->a;
    const double wb = (q & 2) ? t->b : 1.0 - t->b;
    return wa * wb;
}

static void mm_tap_dw(const mm_taps* t, int q, double* dX, double* dY)
{
    const double wa = (q & 1) ? t->a : 1.0 - t->a;
    const double wb = (q & 2) ? t->b : 1.0 - t->b;
    *dX = (q & 1) ? wb : -wb;
    *dY = (q & 2) ? wa : -wa;
}

static void mm_tap_flows(const mm_win* w, int f, const mm_taps* t, d2 uq[4])
{
    for (int q = 0; q < 4; ++q) {
        if (mm_tap_in(t, q)) uq[q] = mm_flow(w, f, t->x0 + (q & 1), t->y0 + (q >> 1));
        else { uq[q].x = 0.0; uq[q].y = 0.0; }
    }
}

static int mm_inside(const mm_win* w, double X, double Y)
{
    return X >= 0.0 && X <= w->xmax && Y >= 0.0 && Y <= w->ymax;
}

static int mm_refs_before(const mm_win* w, double t)
{
    int m = 0;
    for (int r = 0; r < w->R; ++r) m += w->refs[r] < t;
    return m;
}

/* The warp; px/py indexed by reference.  Returns validity, *mb = refs before t. */
static int mm_warp(const mm_win* w, double x0, double y0, double tk, double* px, double* py, int* mbo)
{
    *mbo = 0;
    if (!(isfinite(x0) && isfinite(y0) && tk >= 0.0 && tk <= 1.0 && mm_inside(w, x0, y0))) return 0;
    const int mb = mm_refs_before(w, tk);
    *mbo = mb;
    int rs = mb;
    if (rs < w->R && w->refs[rs] == tk) { px[rs] = x0; py[rs] = y0; ++rs; }
    const int nf = w->R - rs, nv = nf + mb;
    double X = x0, Y = y0, tau = tk;
    for (int j = 0; j < nv; ++j) {
        int r, f;
        if (j < nf) { r = rs + j; f = w->sf[r]; }
        else {
            r = mb - 1 - (j - nf);
            f = w->sb[r];
            if (j == nf) { X = x0; Y = y0; tau = tk; }
        }
        const mm_taps t = mm_make_taps(w, X, Y);
        d2 uq[4];
        mm_tap_flows(w, f, &t, uq);
        double ux = 0.0, uy = 0.0;
        for (int q = 0; q < 4; ++q) {
            const double wq = mm_tap_w(&t, q);
            ux += wq * uq[q].x;
            uy += wq * uq[q].y;
        }
        const double ref = w->refs[r];
        const double dt = ref - tau;
        X = X + dt * ux;
        Y = Y + dt * uy;
        tau = ref;
        if (!mm_inside(w, X, Y)) return 0;
        px[r] = X; py[r] = Y;
    }
    return 1;
}

static int mm_tile_of(const mm_win* w, double X, double Y)
{
    const mm_taps t = mm_make_taps(w, X, Y);
    return (t.y0 / TH) * w->ntx + t.x0 / TW;
}

/* ------------------------------------------------------------------------
 * Reductions in the GPU's order
 * ---------------------------------------------------------------------- */

/* Lane 0 of a 64-lane shuffle-down tree. */
static double mm_wave_sum(double* v)
{
    for (int o = 32; o > 0; o >>= 1)
        for (int l = 0; l < o; ++l) v[l] = v[l] + v[l + o];
    return v[0];
}

/* Block of nthreads (multiple of 64): per-wavefront trees, then the wave
 * results in order. */
static double mm_block_sum(double* v, int nthreads)
{
    double s = 0.0;
    for (int wv = 0; wv < nthreads / 64; ++wv) {
        const double ws = mm_wave_sum(v + 64 * wv);
        s += ws;
    }
    return s;
}

static void mm_reduce_pixel(d2 a, d2 b, double eps, double* sum, double* cnt)
{
    if (a.x + b.x > 0.0) *cnt += 1.0;
    if (a.x != 0.0 || a.y != 0.0) { const double T = a.y / (a.x + eps); *sum += T * T; }
    if (b.x != 0.0 || b.y != 0.0) { const double T = b.y / (b.x + eps); *sum += T * T; }
}

/* ------------------------------------------------------------------------
 * Forward
 * ---------------------------------------------------------------------- */

typedef struct { double X, Y; float t; int neg; } mm_srec;

typedef struct {
    mm_win w;
    d2* img;           /* [R][2][HW] */
    double num[MM_MAX_REFS], nact[MM_MAX_REFS];
    double loss;
    uint64_t n_valid;
} mm_state;

static int mm_forward_impl(mm_state* S, int64_t n, const float* ex, const float* ey,
                           const float* et, const int8_t* ep)
{
    mm_win* w = &S->w;
    const int R = w->R, nbins = R * w->ntiles;
    /* records in canonical order: events in order, then references */
    int64_t* cnt = (int64_t*)calloc((size_t)nbins + 1, sizeof(int64_t));
    double px[MM_MAX_REFS], py[MM_MAX_REFS];
    int mb;
    S->n_valid = 0;
    for (int64_t k = 0; k < n; ++k) {
        if (!mm_warp(w, ex[k], ey[k], et[k], px, py, &mb)) continue;
        ++S->n_valid;
        for (int r = 0; r < R; ++r) cnt[r * w->ntiles + mm_tile_of(w, px[r], py[r]) + 1]++;
    }
    for (int b = 0; b < nbins; ++b) cnt[b + 1] += cnt[b];
    mm_srec* rec = (mm_srec*)malloc(sizeof(mm_srec) * (size_t)(cnt[nbins] + 1));
    int64_t* fill = (int64_t*)malloc(sizeof(int64_t) * (size_t)nbins);
    if (!rec || !fill) { free(cnt); free(rec); free(fill); return MM_NOMEM; }
    memcpy(fill, cnt, sizeof(int64_t) * (size_t)nbins);
    for (int64_t k = 0; k < n; ++k) {
        if (!mm_warp(w, ex[k], ey[k], et[k], px, py, &mb)) continue;
        for (int r = 0; r < R; ++r) {
            const int b = r * w->ntiles + mm_tile_of(w, px[r], py[r]);
            mm_srec* q = &rec[fill[b]++];
            q->X = px[r]; q->Y = py[r]; q->t = et[k]; q->neg = !(ep[k] > 0);
        }
    }
    free(fill);

    S->img = (d2*)calloc((size_t)R * 2 * w->HW, sizeof(d2));
    d2* halo = (d2*)calloc((size_t)nbins * NHALO * 2, sizeof(d2));
    double* part = (double*)calloc((size_t)nbins * 4, sizeof(double));
    d2* lds = (d2*)malloc(sizeof(d2) * 2 * TLW * TLH);
    double* red = (double*)malloc(sizeof(double) * 256);
    double* red2 = (double*)malloc(sizeof(double) * 256);
    if (!S->img || !halo || !part || !lds || !red || !red2) return MM_NOMEM;

    for (int b = 0; b < nbins; ++b) {
        const int r = b / w->ntiles, tile = b - r * w->ntiles;
        const int ty = tile / w->ntx, tx = tile - ty * w->ntx;
        const int xo = tx * TW, yo = ty * TH;
        const double ref = w->refs[r];
        memset(lds, 0, sizeof(d2) * 2 * TLW * TLH);
        for (int64_t c0 = cnt[b]; c0 < cnt[b + 1]; c0 += 64) {
            const int64_t c1 = c0 + 64 < cnt[b + 1] ? c0 + 64 : cnt[b + 1];
            for (int q = 0; q < 4; ++q)
                for (int64_t i = c0; i < c1; ++i) {
                    const mm_srec* s = &rec[i];
                    const mm_taps tp = mm_make_taps(w, s->X, s->Y);
                    const double wt = mm_tap_w(&tp, q);
                    if (!(mm_tap_in(&tp, q) && wt != 0.0)) continue;
                    const double tb = 1.0 - fabs(ref - (double)s->t);
                    const int key = (s->neg ? TLW * TLH : 0) + (tp.y0 - yo + (q >> 1)) * TLW +
                                    tp.x0 - xo + (q & 1);
                    lds[key].x = lds[key].x + wt;
                    lds[key].y = lds[key].y + wt * tb;
                }
        }
        /* own pixels + interior reduce (256 threads, pixel i to thread i % 256) */
        for (int th = 0; th < 256; ++th) { red[th] = 0.0; red2[th] = 0.0; }
        for (int i = 0; i < TW * TH; ++i) {
            const int lx = i % TW, ly = i / TW, X = xo + lx, Y = yo + ly;
            if (X >= w->W || Y >= w->H) continue;
            const d2 a = lds[ly * TLW + lx], c = lds[TLW * TLH + ly * TLW + lx];
            S->img[(size_t)(r * 2 + 0) * w->HW + Y * w->W + X] = a;
            S->img[(size_t)(r * 2 + 1) * w->HW + Y * w->W + X] = c;
            if (lx > 0 && ly > 0) mm_reduce_pixel(a, c, w->eps, &red[i % 256], &red2[i % 256]);
        }
        d2* hb = halo + (size_t)b * NHALO * 2;
        for (int j = 0; j < NHALO; ++j) {
            const int idx = (j <= TH) ? j * TLW + TW : TH * TLW + (j - (TH + 1));
            hb[j * 2 + 0] = lds[idx];
            hb[j * 2 + 1] = lds[TLW * TLH + idx];
        }
        part[(b * 2 + 0) * 2 + 0] = mm_block_sum(red, 256);
        part[(b * 2 + 0) * 2 + 1] = mm_block_sum(red2, 256);
    }
    /* merge (64 threads, border pixel j to thread j) */
    for (int b = 0; b < nbins; ++b) {
        const int r = b / w->ntiles, tile = b - r * w->ntiles;
        const int ty = tile / w->ntx, tx = tile - ty * w->ntx;
        const int xo = tx * TW, yo = ty * TH;
        for (int th = 0; th < 64; ++th) { red[th] = 0.0; red2[th] = 0.0; }
        for (int j = 0; j < NBORDER; ++j) {
            const int lx = j < TH ? 0 : j - TH + 1, ly = j < TH ? j : 0;
            const int X = xo + lx, Y = yo + ly;
            if (X >= w->W || Y >= w->H) continue;
            const int pix = Y * w->W + X;
            d2 v[2];
            for (int pol = 0; pol < 2; ++pol) {
                d2 a = S->img[(size_t)(r * 2 + pol) * w->HW + pix];
                if (lx == 0 && tx > 0) {
                    const d2 h = halo[((size_t)(b - 1) * NHALO + ly) * 2 + pol];
                    a.x += h.x; a.y += h.y;
                }
                if (ly == 0 && ty > 0) {
                    const d2 h = halo[((size_t)(b - w->ntx) * NHALO + TH + 1 + lx) * 2 + pol];
                    a.x += h.x; a.y += h.y;
                }
                if (lx == 0 && ly == 0 && tx > 0 && ty > 0) {
                    const d2 h = halo[((size_t)(b - w->ntx - 1) * NHALO + TH) * 2 + pol];
                    a.x += h.x; a.y += h.y;
                }
                S->img[(size_t)(r * 2 + pol) * w->HW + pix] = a;
                v[pol] = a;
            }
            mm_reduce_pixel(v[0], v[1], w->eps, &red[j % 64], &red2[j % 64]);
        }
        part[(b * 2 + 1) * 2 + 0] = mm_block_sum(red, 64);
        part[(b * 2 + 1) * 2 + 1] = mm_block_sum(red2, 64);
    }
    /* finalize (256 threads) */
    double L = 0.0;
    for (int r = 0; r < R; ++r) {
        for (int th = 0; th < 256; ++th) { red[th] = 0.0; red2[th] = 0.0; }
        for (int j = 0; j < 2 * w->ntiles; ++j) {
            red[j % 256] += part[((size_t)r * 2 * w->ntiles + j) * 2 + 0];
            red2[j % 256] += part[((size_t)r * 2 * w->ntiles + j) * 2 + 1];
        }
        const double s = mm_block_sum(red, 256), c = mm_block_sum(red2, 256);
        S->num[r] = s;
        S->nact[r] = c;
        L += s / (c + w->eps);
    }
    S->loss = L / (double)R;
    free(cnt); free(rec); free(halo); free(part); free(lds); free(red); free(red2);
    return MM_OK;
}

int cmm_forward(int W, int H, const float* K, int R, const float* refs, float eps, int F,
                int model, int64_t n, const float* x, const float* y, const float* t, const int8_t* p,
                const float* rho, const float* theta, float* loss_out, double* hdr_out)
{
    mm_state S;
    memset(&S, 0, sizeof S);
    if (mm_setup(&S.w, W, H, K, R, refs, eps, F, model, rho, theta, n)) return MM_BAD;
    const int st = mm_forward_impl(&S, n, x, y, t, p);
    if (st == MM_OK) {
        *loss_out = (float)S.loss;
        if (hdr_out) {
            hdr_out[0] = S.loss;
            hdr_out[1] = (double)S.n_valid;
            for (int r = 0; r < R; ++r) { hdr_out[2 + r] = S.num[r]; hdr_out[2 + R + r] = S.nact[r]; }
        }
    }
    free(S.img);
    return st;
}

/* ------------------------------------------------------------------------
 * Backward
 * ---------------------------------------------------------------------- */

typedef struct { double X, Y, gx, gy; } mm_grec;

/* The direct sensitivity (seed) of one reference position, added into L. */
static void mm_direct(const mm_win* w, const d2* plane, double coef, double tb, double X, double Y,
                      double* Lx, double* Ly)
{
    const mm_taps tp = mm_make_taps(w, X, Y);
    for (int q = 0; q < 4; ++q) {
        if (!mm_tap_in(&tp, q)) continue;
        const d2 cs = plane[(tp.y0 + (q >> 1)) * w->W + tp.x0 + (q & 1)];
        const double S = cs.y;
        const double inv = 1.0 / (cs.x + w->eps);
        const double sc = S * inv;
        const double g = coef * sc * inv * (tb - sc);
        double dX, dY;
        mm_tap_dw(&tp, q, &dX, &dY);
        *Lx += g * dX;
        *Ly += g * dY;
    }
}

static void mm_jacobian_t(const mm_win* w, int f, double X, double Y, double Lx, double Ly,
                          double* jx, double* jy)
{
    const mm_taps tp = mm_make_taps(w, X, Y);
    d2 uq[4];
    mm_tap_flows(w, f, &tp, uq);
    *jx = 0.0;
    *jy = 0.0;
    for (int q = 0; q < 4; ++q) {
        const double lu = Lx * uq[q].x + Ly * uq[q].y;
        double dX, dY;
        mm_tap_dw(&tp, q, &dX, &dY);
        *jx += lu * dX;
        *jy += lu * dY;
    }
}

static void mm_dtheta(const mm_win* w, int i, int j, double r, double gx, double gy, double* dth)
{
    const double xb = (double)i - w->cx, yb = (double)j - w->cy;
    dth[0] += r * w->fx * gx;
    dth[1] += r * w->fy * gy;
    dth[2] -= r * (xb * gx + yb * gy);
    dth[3] -= (xb * yb * w->inv_fy) * gx + (w->fy + yb * yb * w->inv_fy) * gy;
    dth[4] += (w->fx + xb * xb * w->inv_fx) * gx + (xb * yb * w->inv_fx) * gy;
    dth[5] += (w->fy_over_fx * xb) * gy - (w->fx_over_fy * yb) * gx;
}

/* d rho of dL/du = (gx, gy) at pixel (i, j) of set f; the pixel's d theta
 * share is added into dth (both models) */
static double mm_chain(const mm_win* w, int f, int i, int j, double r, double gx, double gy,
                       double* dth)
{
    if (w->model == 1) {
        double xn, yn, p[3];
        mm_point(w, f, i, j, r, &xn, &yn, p);
        if (!(p[2] > 0.0)) return 0.0;
        const double* Rm = w->Rm[f];
        const double* v = w->v[f];
        const double* Jr = w->Jr[f];
        const double iz = 1.0 / p[2];
        const double ax = gx * w->fx, ay = gy * w->fy;
        const double q[3] = {ax * iz, ay * iz, -((ax * p[0] + ay * p[1]) * iz) * iz};
        const double drho = (q[0] * v[0] + q[1] * v[1]) + q[2] * v[2];
        for (int k = 0; k < 3; ++k) dth[k] += r * q[k];
        double sv[3];
        for (int k = 0; k < 3; ++k) sv[k] = (Rm[k] * q[0] + Rm[3 + k] * q[1]) + Rm[6 + k] * q[2];
        const double c[3] = {yn * sv[2] - sv[1], sv[0] - xn * sv[2], xn * sv[1] - yn * sv[0]};
        for (int k = 0; k < 3; ++k) dth[3 + k] += (Jr[k] * c[0] + Jr[3 + k] * c[1]) + Jr[6 + k] * c[2];
        return drho;
    }
    double Ax, Ay, Bx, By;
    mm_parts(w, f, i, j, &Ax, &Ay, &Bx, &By);
    if (gx != 0.0 || gy != 0.0) mm_dtheta(w, i, j, r, gx, gy, dth);
    return gx * Bx + gy * By;
}

/* One wavefront-iteration of the sweep: the per-lane reverse passes run in
 * lockstep; records are emitted at each program point in lane order. */
typedef struct {
    int live, nv, rs, mb, pol;
    double x0, y0, tk, px[MM_MAX_REFS], py[MM_MAX_REFS];
    double Lx, Ly, g0x, g0y;
} mm_lane;

static void mm_emit(const mm_win* w, mm_grec* rec, int64_t* fill, int f, double X, double Y,
                    double gx, double gy)
{
    mm_grec* q = &rec[fill[f * w->ntiles + mm_tile_of(w, X, Y)]++];
    q->X = X; q->Y = Y; q->gx = gx; q->gy = gy;
}

int cmm_backward(int W, int H, const float* K, int R, const float* refs, float eps, int F,
                 int model, int64_t n, const float* x, const float* y, const float* t, const int8_t* p,
                 const float* rho, const float* theta, float grad_loss, float* drho_out,
                 float* dtheta_out)
{
    mm_state S;
    memset(&S, 0, sizeof S);
    if (mm_setup(&S.w, W, H, K, R, refs, eps, F, model, rho, theta, n)) return MM_BAD;
    int st = mm_forward_impl(&S, n, x, y, t, p);
    if (st) { free(S.img); return st; }
    const mm_win* w = &S.w;
    const int nt = w->ntiles, nbb = F * nt;
    const int split = F > 1;     /* one record per first step (else one per event) */
    double coef[MM_MAX_REFS];
    for (int r = 0; r < R; ++r) coef[r] = w->two_over_R / (S.nact[r] + w->eps);

    /* count: sampling positions per (flow set, tile) bin */
    int64_t* cnt = (int64_t*)calloc((size_t)nbb + 1, sizeof(int64_t));
    double px[MM_MAX_REFS], py[MM_MAX_REFS];
    int mb;
    for (int64_t k = 0; k < n; ++k) {
        if (!mm_warp(w, x[k], y[k], t[k], px, py, &mb)) continue;
        const int rs = (mb < R && w->refs[mb] == (double)t[k]) ? mb + 1 : mb;
        if (split) {
            for (int r = rs; r < R; ++r) {
                const double X = r == rs ? x[k] : px[r - 1], Y = r == rs ? y[k] : py[r - 1];
                cnt[w->sf[r] * nt + mm_tile_of(w, X, Y) + 1]++;
            }
            for (int r = mb - 1; r >= 0; --r) {
                const double X = r == mb - 1 ? x[k] : px[r + 1];
                const double Y = r == mb - 1 ? y[k] : py[r + 1];
                cnt[w->sb[r] * nt + mm_tile_of(w, X, Y) + 1]++;
            }
        } else {
            for (int r = rs + 1; r < R; ++r) cnt[mm_tile_of(w, px[r - 1], py[r - 1]) + 1]++;
            for (int r = mb - 2; r >= 0; --r) cnt[mm_tile_of(w, px[r + 1], py[r + 1]) + 1]++;
            if (rs < R || mb > 0) cnt[mm_tile_of(w, x[k], y[k]) + 1]++;
        }
    }
    for (int b = 0; b < nbb; ++b) cnt[b + 1] += cnt[b];
    mm_grec* rec = (mm_grec*)malloc(sizeof(mm_grec) * (size_t)(cnt[nbb] + 1));
    int64_t* fill = (int64_t*)malloc(sizeof(int64_t) * (size_t)nbb);
    memcpy(fill, cnt, sizeof(int64_t) * (size_t)nbb);

    /* source order: the valid events grouped by the tile of their position
     * at reference 0, in event order within a tile (the forward's reference-0
     * record order) */
    int64_t* tcnt = (int64_t*)calloc((size_t)nt + 1, sizeof(int64_t));
    int64_t nvalid = 0;
    for (int64_t k = 0; k < n; ++k) {
        if (!mm_warp(w, x[k], y[k], t[k], px, py, &mb)) continue;
        tcnt[mm_tile_of(w, px[0], py[0]) + 1]++;
        ++nvalid;
    }
    for (int b = 0; b < nt; ++b) tcnt[b + 1] += tcnt[b];
    int64_t* order = (int64_t*)malloc(sizeof(int64_t) * (size_t)(nvalid + 1));
    for (int64_t k = 0; k < n; ++k) {
        if (!mm_warp(w, x[k], y[k], t[k], px, py, &mb)) continue;
        order[tcnt[mm_tile_of(w, px[0], py[0])]++] = k;
    }
    free(tcnt);

    /* sweep: in iteration e, block b takes the source positions
     * [(e * nblocks + b) * 64, +64), its 64 lanes in lockstep over the visits
     * j = R-1 .. 0 (the backward sweep backwards, then the forward sweep
     * backwards); the records of one visit number are emitted in lane order,
     * then (one flow set) the event records in lane order. */
    mm_lane lanes[64];
    for (int blk = 0; blk < w->nblocks; ++blk) {
        for (int e = 0; e < w->ept; ++e) {
            for (int l = 0; l < 64; ++l) {
                mm_lane* L = &lanes[l];
                const int64_t i = ((int64_t)e * w->nblocks + blk) * 64 + l;
                L->live = 0;
                if (i >= nvalid) continue;
                const int64_t k = order[i];
                if (!mm_warp(w, x[k], y[k], t[k], L->px, L->py, &L->mb)) continue;
                L->live = 1;
                L->x0 = x[k]; L->y0 = y[k]; L->tk = t[k];
                L->pol = p[k] > 0 ? 0 : 1;
                L->rs = (L->mb < R && w->refs[L->mb] == L->tk) ? 1 : 0;   /* eq */
                L->nv = R - L->mb;                                       /* nf */
                L->Lx = L->Ly = L->g0x = L->g0y = 0.0;
            }
            for (int j = R - 1; j >= 0; --j) {
                for (int l = 0; l < 64; ++l) {
                    mm_lane* L = &lanes[l];
                    if (!L->live) continue;
                    const int nf = L->nv, eq = L->rs, jf = eq ? 1 : 0;
                    if (eq && j == 0) continue;                     /* no step */
                    const int first = (j == jf && j < nf) || (j == nf);
                    const int restart = (j == R - 1) || (j == nf - 1);
                    const int r = j < nf ? L->mb + j : L->mb - 1 - (j - nf);
                    const int f = j < nf ? w->sf[r] : w->sb[r];
                    int rp = r;
                    if (j > 0) rp = (j - 1) < nf ? L->mb + (j - 1) : L->mb - 1 - (j - 1 - nf);
                    const double X = first ? L->x0 : L->px[rp];
                    const double Y = first ? L->y0 : L->py[rp];
                    const double dt = w->refs[r] - ((first || j == 0) ? L->tk : w->refs[rp]);
                    if (restart) { L->Lx = 0.0; L->Ly = 0.0; }
                    mm_direct(w, S.img + (size_t)(r * 2 + L->pol) * w->HW, coef[r],
                              1.0 - fabs(w->refs[r] - L->tk), L->px[r], L->py[r], &L->Lx, &L->Ly);
                    if (first) {
                        if (split) {
                            mm_emit(w, rec, fill, f, L->x0, L->y0, dt * L->Lx, dt * L->Ly);
                        } else {
                            L->g0x += dt * L->Lx;
                            L->g0y += dt * L->Ly;
                        }
                    } else {
                        mm_emit(w, rec, fill, f, X, Y, dt * L->Lx, dt * L->Ly);
                        double jx, jy;
                        mm_jacobian_t(w, f, X, Y, L->Lx, L->Ly, &jx, &jy);
                        L->Lx += dt * jx;
                        L->Ly += dt * jy;
                    }
                }
            }
            for (int l = 0; l < 64; ++l) {
                mm_lane* L = &lanes[l];
                if (!split && L->live && R - (L->rs ? 1 : 0) > 0)
                    mm_emit(w, rec, fill, 0, L->x0, L->y0, L->g0x, L->g0y);
            }
        }
    }
    free(fill);
    free(order);

    /* tiles, per (flow set, tile) bin: dL/du in LDS order, then d rho and
     * d theta shares of that set */
    const double gl = (double)grad_loss;
    d2* halo = (d2*)calloc((size_t)nbb * NHALO, sizeof(d2));
    d2* border = (d2*)calloc((size_t)nbb * NBORDER, sizeof(d2));
    double* part = (double*)calloc((size_t)nbb * 12, sizeof(double));
    d2* lds = (d2*)malloc(sizeof(d2) * TLW * TLH);
    double* red = (double*)malloc(sizeof(double) * 256 * 6);
    for (int b = 0; b < nbb; ++b) {
        const int f = b / nt, tile = b - f * nt;
        const int ty = tile / w->ntx, tx = tile - ty * w->ntx;
        const int xo = tx * TW, yo = ty * TH;
        const float* rho_f = rho + (size_t)f * w->HW;
        float* drho_f = drho_out + (size_t)f * w->HW;
        memset(lds, 0, sizeof(d2) * TLW * TLH);
        for (int64_t c0 = cnt[b]; c0 < cnt[b + 1]; c0 += 64) {
            const int64_t c1 = c0 + 64 < cnt[b + 1] ? c0 + 64 : cnt[b + 1];
            for (int q = 0; q < 4; ++q)
                for (int64_t i = c0; i < c1; ++i) {
                    const mm_grec* s = &rec[i];
                    const mm_taps tp = mm_make_taps(w, s->X, s->Y);
                    const double wt = mm_tap_w(&tp, q);
                    if (!(mm_tap_in(&tp, q) && wt != 0.0)) continue;
                    const int key = (tp.y0 - yo + (q >> 1)) * TLW + tp.x0 - xo + (q & 1);
                    lds[key].x = lds[key].x + wt * s->gx;
                    lds[key].y = lds[key].y + wt * s->gy;
                }
        }
        memset(red, 0, sizeof(double) * 256 * 6);
        for (int i = 0; i < TW * TH; ++i) {
            const int lx = i % TW, ly = i / TW, X = xo + lx, Y = yo + ly;
            if (X >= w->W || Y >= w->H) continue;
            const d2 g = lds[ly * TLW + lx];
            if (lx == 0 || ly == 0) {
                border[(size_t)b * NBORDER + (lx == 0 ? ly : TH + lx - 1)] = g;
                continue;
            }
            const int pix = Y * w->W + X;
            double d[6];
            for (int c = 0; c < 6; ++c) d[c] = red[c * 256 + i % 256];
            double dr = 0.0;
            if (w->model == 0 || g.x != 0.0 || g.y != 0.0)
                dr = mm_chain(w, f, X, Y, (double)rho_f[pix], g.x, g.y, d);
            drho_f[pix] = (float)(gl * dr);
            for (int c = 0; c < 6; ++c) red[c * 256 + i % 256] = d[c];
        }
        for (int j = 0; j < NHALO; ++j) {
            const int idx = (j <= TH) ? j * TLW + TW : TH * TLW + (j - (TH + 1));
            halo[(size_t)b * NHALO + j] = lds[idx];
        }
        for (int c = 0; c < 6; ++c) part[(size_t)b * 12 + c] = mm_block_sum(red + c * 256, 256);
    }
    for (int b = 0; b < nbb; ++b) {
        const int f = b / nt, tile = b - f * nt;
        const int ty = tile / w->ntx, tx = tile - ty * w->ntx;
        const int xo = tx * TW, yo = ty * TH;
        const float* rho_f = rho + (size_t)f * w->HW;
        float* drho_f = drho_out + (size_t)f * w->HW;
        memset(red, 0, sizeof(double) * 64 * 6);
        for (int j = 0; j < NBORDER; ++j) {
            const int lx = j < TH ? 0 : j - TH + 1, ly = j < TH ? j : 0;
            const int X = xo + lx, Y = yo + ly;
            if (X >= w->W || Y >= w->H) continue;
            d2 g = border[(size_t)b * NBORDER + j];
            if (lx == 0 && tx > 0) {
                const d2 h = halo[(size_t)(b - 1) * NHALO + ly];
                g.x += h.x; g.y += h.y;
            }
            if (ly == 0 && ty > 0) {
                const d2 h = halo[(size_t)(b - w->ntx) * NHALO + TH + 1 + lx];
                g.x += h.x; g.y += h.y;
            }
            if (lx == 0 && ly == 0 && tx > 0 && ty > 0) {
                const d2 h = halo[(size_t)(b - w->ntx - 1) * NHALO + TH];
                g.x += h.x; g.y += h.y;
            }
            const int pix = Y * w->W + X;
            double d[6];
            for (int c = 0; c < 6; ++c) d[c] = red[c * 64 + j % 64];
            double dr = 0.0;
            if (w->model == 0 || g.x != 0.0 || g.y != 0.0)
                dr = mm_chain(w, f, X, Y, (double)rho_f[pix], g.x, g.y, d);
            drho_f[pix] = (float)(gl * dr);
            for (int c = 0; c < 6; ++c) red[c * 64 + j % 64] = d[c];
        }
        for (int c = 0; c < 6; ++c) part[(size_t)b * 12 + 6 + c] = mm_block_sum(red + c * 64, 64);
    }
    /* finalize per flow set (256 threads) */
    for (int f = 0; f < F; ++f)
        for (int c = 0; c < 6; ++c) {
            memset(red, 0, sizeof(double) * 256);
            const double* pf = part + (size_t)f * nt * 12;
            for (int j = 0; j < 2 * nt; ++j) red[j % 256] += pf[(size_t)j * 6 + c];
            dtheta_out[f * 6 + c] = (float)(gl * mm_block_sum(red, 256));
        }
    free(cnt); free(rec); free(halo); free(border); free(part); free(lds); free(red); free(S.img);
    return MM_OK;
}
