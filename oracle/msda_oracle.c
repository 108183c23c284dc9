/*
 * FP64 CPU oracle for multi-scale deformable aggregation (MSDA).
 *
 * TEST INFRASTRUCTURE ONLY. This file is the correctness authority that the
 * HIP kernels are checked against. Only the tests, the smoke check and the
 * benchmark's CPU-baseline leg may load it; the product path never does. It
 * shares no code, header or constant with the GPU library.
 *
 * What it computes (paper Sec. 3.1 and Sec. 3.2: every 3D anchor's keypoints
 * are projected into each camera, the camera's multi-scale feature maps are
 * sampled at the projected point, and the samples are aggregated; Sec. 5.3
 * names the operator). MSDA has a plain closed-form definition, so this is
 * that definition written out with loops, in double precision:
 *
 *   for every batch item b, anchor a, keypoint p, camera n, level l:
 *     (H, W) = spatial_shapes[n][l], s0 = level_start_index[n][l]
 *     (u, v) = sampling_loc[b][a][p][n]            (normalised, 0..1 = image)
 *     x = u*W - 0.5, y = v*H - 0.5                 (pixel centres at i + 0.5)
 *     skip unless -1 < x < W and -1 < y < H
 *     bilinear value val[c] over the 4 integer neighbours of (x, y), a corner
 *       outside the level contributing zero
 *     out[b][a][c] += weights[b][a][p][n][l][c / (C/G)] * val[c]
 *
 * The backward is the analytic derivative of that sum with respect to feat,
 * sampling_loc and weights (chain rule through the bilinear weights; the
 * derivative at an integer coordinate is the right-hand one, the value of
 * floor() there).
 *
 * Threading: OpenMP over independent outputs only; every output element is
 * accumulated by one thread in one fixed order, so results are bitwise
 * independent of the thread count.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct {
    int valid;              /* sample lies in (-1, W) x (-1, H)                */
    double lx, ly;          /* fractional offsets from the top-left neighbour  */
    double cw[4];           /* corner weights, zero for a corner outside       */
    int64_t row[4];         /* feature row of each corner (if inside)          */
    int inside[4];          /* corner inside the level                         */
} sample_t;

/* Corners in the order (y0,x0), (y0,x0+1), (y0+1,x0), (y0+1,x0+1). */
static void locate(double u, double v, int H, int W, int64_t s0, sample_t* s)
{
    const double x = u * (double)W - 0.5;
    const double y = v * (double)H - 0.5;
    memset(s, 0, sizeof(*s));
    s->valid = (x > -1.0) && (y > -1.0) && (x < (double)W) && (y < (double)H);
    if (!s->valid) return;
    const double fx = floor(x), fy = floor(y);
    const int x0 = (int)fx, y0 = (int)fy;
    s->lx = x - fx;
    s->ly = y - fy;
    const double hx = 1.0 - s->lx, hy = 1.0 - s->ly;
    const int cx[4] = {x0, x0 + 1, x0, x0 + 1};
    const int cy[4] = {y0, y0, y0 + 1, y0 + 1};
    const double w4[4] = {hy * hx, hy * s->lx, s->ly * hx, s->ly * s->lx};
    for (int k = 0; k < 4; ++k) {
        s->inside[k] = (cx[k] >= 0) && (cx[k] < W) && (cy[k] >= 0) && (cy[k] < H);
        s->cw[k] = s->inside[k] ? w4[k] : 0.0;
        s->row[k] = s->inside[k] ? s0 + (int64_t)cy[k] * W + cx[k] : -1;
    }
}

static void set_threads(int nthreads)
{
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
}

int msda_oracle_num_threads(void)
{
#ifdef _OPENMP
    int n = 1;
#pragma omp parallel
    {
#pragma omp single
        n = omp_get_num_threads();
    }
    return n;
#else
    return 1;
#endif
}

/*
 * out[B][A][C] = sum over (p, n, l) of weights * bilinear(feat).
 * feat [B][R][C], spatial_shapes [N][L][2] (H, W), level_start_index [N][L],
 * sampling_loc [B][A][P][N][2], weights [B][A][P][N][L][G].
 */
void msda_oracle_forward(int B, int N, int L, int A, int P, int C, int G, int64_t R,
                         const double* feat, const int32_t* spatial_shapes,
                         const int32_t* level_start_index, const double* sampling_loc,
                         const double* weights, double* out, int nthreads)
{
    set_threads(nthreads);
    const int cpg = C / G;
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t ba = 0; ba < (int64_t)B * A; ++ba) {
        const int b = (int)(ba / A);
        double* o = out + ba * C;
        for (int c = 0; c < C; ++c) o[c] = 0.0;
        for (int p = 0; p < P; ++p) {
            for (int n = 0; n < N; ++n) {
                const double* uv = sampling_loc + (((ba * P) + p) * N + n) * 2;
                for (int l = 0; l < L; ++l) {
                    const int H = spatial_shapes[(n * L + l) * 2 + 0];
                    const int W = spatial_shapes[(n * L + l) * 2 + 1];
                    sample_t s;
                    locate(uv[0], uv[1], H, W, level_start_index[n * L + l], &s);
                    if (!s.valid) continue;
                    const double* w = weights + ((((ba * P) + p) * N + n) * L + l) * G;
                    for (int c = 0; c < C; ++c) {
                        double val = 0.0;
                        for (int k = 0; k < 4; ++k)
                            if (s.inside[k])
                                val += s.cw[k] * feat[((int64_t)b * R + s.row[k]) * C + c];
                        o[c] += w[c / cpg] * val;
                    }
                }
            }
        }
    }
}

/* 1 when the (n, l) regions of a batch item are pairwise disjoint. */
static int regions_disjoint(int N, int L, const int32_t* shapes, const int32_t* starts)
{
    const int m = N * L;
    for (int i = 0; i < m; ++i) {
        const int64_t a0 = starts[i], a1 = a0 + (int64_t)shapes[2 * i] * shapes[2 * i + 1];
        for (int j = i + 1; j < m; ++j) {
            const int64_t b0 = starts[j], b1 = b0 + (int64_t)shapes[2 * j] * shapes[2 * j + 1];
            if (a0 < b1 && b0 < a1) return 0;
        }
    }
    return 1;
}

/*
 * Gradients of loss = <grad_out, out>. Any output pointer may be NULL to skip it.
 *   grad_feat [B][R][C]: sum of corner weight * weight * grad_out over every
 *                        sample touching a row (rows no sample touches are 0);
 *   grad_loc  [B][A][P][N][2]: sum over levels of W (resp. H) times the
 *                        derivative of the weighted bilinear value along x (y);
 *   grad_w    [B][A][P][N][L][G]: <grad_out, val> over the group's channels.
 * Skipped (out-of-range) samples contribute nothing anywhere.
 */
void msda_oracle_backward(int B, int N, int L, int A, int P, int C, int G, int64_t R,
                          const double* feat, const int32_t* spatial_shapes,
                          const int32_t* level_start_index, const double* sampling_loc,
                          const double* weights, const double* grad_out,
                          double* grad_feat, double* grad_loc, double* grad_w, int nthreads)
{
    set_threads(nthreads);
    const int cpg = C / G;

    if (grad_loc || grad_w) {
#pragma omp parallel for schedule(dynamic, 4)
        for (int64_t ba = 0; ba < (int64_t)B * A; ++ba) {
            const int b = (int)(ba / A);
            const double* go = grad_out + ba * C;
            for (int p = 0; p < P; ++p) {
                for (int n = 0; n < N; ++n) {
                    const int64_t pn = (ba * P + p) * N + n;
                    const double* uv = sampling_loc + pn * 2;
                    double gx = 0.0, gy = 0.0;
                    for (int l = 0; l < L; ++l) {
                        const int H = spatial_shapes[(n * L + l) * 2 + 0];
                        const int W = spatial_shapes[(n * L + l) * 2 + 1];
                        const double* w = weights + (pn * L + l) * G;
                        double* gw = grad_w ? grad_w + (pn * L + l) * G : NULL;
                        if (gw) for (int g = 0; g < G; ++g) gw[g] = 0.0;
                        sample_t s;
                        locate(uv[0], uv[1], H, W, level_start_index[n * L + l], &s);
                        if (!s.valid) continue;
                        const double hx = 1.0 - s.lx, hy = 1.0 - s.ly;
                        double dx_sum = 0.0, dy_sum = 0.0;
                        for (int c = 0; c < C; ++c) {
                            double f[4];
                            for (int k = 0; k < 4; ++k)
                                f[k] = s.inside[k] ? feat[((int64_t)b * R + s.row[k]) * C + c] : 0.0;
                            const double val = s.cw[0] * f[0] + s.cw[1] * f[1] + s.cw[2] * f[2] +
                                               s.cw[3] * f[3];
                            /* d val / dx and d val / dy inside the cell */
                            const double dvdx = hy * (f[1] - f[0]) + s.ly * (f[3] - f[2]);
                            const double dvdy = hx * (f[2] - f[0]) + s.lx * (f[3] - f[1]);
                            const double wg = w[c / cpg] * go[c];
                            if (gw) gw[c / cpg] += go[c] * val;
                            dx_sum += wg * dvdx;
                            dy_sum += wg * dvdy;
                        }
                        /* x = u*W - 0.5 so dx/du = W; likewise dy/dv = H */
                        gx += (double)W * dx_sum;
                        gy += (double)H * dy_sum;
                    }
                    if (grad_loc) {
                        grad_loc[pn * 2 + 0] = gx;
                        grad_loc[pn * 2 + 1] = gy;
                    }
                }
            }
        }
    }

    if (grad_feat) {
        memset(grad_feat, 0, sizeof(double) * (size_t)B * (size_t)R * (size_t)C);
        /* Camera regions are disjoint in every layout the tests build; then each
         * (b, n) owns its rows and threads never share an element. Otherwise run
         * the same loop serially. The per-element order (a, p, l, corner) is the
         * same either way. */
        const int par = regions_disjoint(N, L, spatial_shapes, level_start_index);
#pragma omp parallel for schedule(dynamic, 1) if (par)
        for (int64_t bn = 0; bn < (int64_t)B * N; ++bn) {
            const int b = (int)(bn / N), n = (int)(bn % N);
            for (int a = 0; a < A; ++a) {
                const int64_t ba = (int64_t)b * A + a;
                const double* go = grad_out + ba * C;
                for (int p = 0; p < P; ++p) {
                    const int64_t pn = (ba * P + p) * N + n;
                    const double* uv = sampling_loc + pn * 2;
                    for (int l = 0; l < L; ++l) {
                        const int H = spatial_shapes[(n * L + l) * 2 + 0];
                        const int W = spatial_shapes[(n * L + l) * 2 + 1];
                        const double* w = weights + (pn * L + l) * G;
                        sample_t s;
                        locate(uv[0], uv[1], H, W, level_start_index[n * L + l], &s);
                        if (!s.valid) continue;
                        for (int k = 0; k < 4; ++k) {
                            if (!s.inside[k]) continue;
                            double* gf = grad_feat + ((int64_t)b * R + s.row[k]) * C;
                            for (int c = 0; c < C; ++c) gf[c] += s.cw[k] * w[c / cpg] * go[c];
                        }
                    }
                }
            }
        }
    }
}

/*
 * Decode OCP FP8 E4M3 ("e4m3fn": 1 sign, 4 exponent bits with bias 7, 3
 * mantissa bits, no infinities, S.1111.111 = NaN, max 448) to double.
 */
void msda_oracle_decode_e4m3(const uint8_t* codes, int64_t n, double* out)
{
    for (int64_t i = 0; i < n; ++i) {
        const unsigned q = codes[i];
        const int sign = (q >> 7) & 1, e = (q >> 3) & 15, m = q & 7;
        double v;
        if (e == 15 && m == 7) v = NAN;
        else if (e == 0) v = ldexp((double)m, -9);          /* subnormal: m/8 * 2^-6 */
        else v = ldexp(8.0 + (double)m, e - 10);            /* (1 + m/8) * 2^(e-7)  */
        out[i] = sign ? -v : v;
    }
}

/*
 * Encode FP32 values to OCP FP8 E4M3 by round-to-nearest-even onto the
 * representable set, after clamping to [-448, 448]. The quotient x / scale is
 * formed in FP32 by the caller (the same precision the kernel divides in);
 * this routine only rounds.
 *
 * The representable magnitudes in [2^e, 2^(e+1)) are spaced 2^(e-3) apart for
 * e >= -6; below 2^-6 (subnormals) the spacing is 2^-9. So the nearest one is
 * rint(v / spacing) * spacing, rint rounding halves to even (the default
 * rounding mode); the division and product are exact powers-of-two scalings.
 */
static unsigned e4m3_code_of(double r)   /* r: a representable magnitude */
{
    if (r == 0.0) return 0;
    if (r < ldexp(1.0, -6)) return (unsigned)(r / ldexp(1.0, -9));      /* e = 0 */
    int ex;
    (void)frexp(r, &ex);                       /* r in [2^(ex-1), 2^ex)       */
    const int e = ex - 1;
    const unsigned m = (unsigned)(r / ldexp(1.0, e - 3)) - 8u;
    return ((unsigned)(e + 7) << 3) | m;
}

void msda_oracle_encode_e4m3(const float* x, int64_t n, uint8_t* codes)
{
    for (int64_t i = 0; i < n; ++i) {
        double v = (double)x[i];
        unsigned sign = 0;
        if (signbit(v)) { sign = 0x80; v = -v; }
        if (v > 448.0) v = 448.0;
        double spacing;
        if (v < ldexp(1.0, -6)) {
            spacing = ldexp(1.0, -9);
        } else {
            int ex;
            (void)frexp(v, &ex);
            spacing = ldexp(1.0, ex - 1 - 3);
        }
        const double r = rint(v / spacing) * spacing;
        codes[i] = (uint8_t)(sign | e4m3_code_of(r));
    }
}

/* The same rounding by exhaustive search over all 127 finite magnitudes
 * (nearest, ties to the even code). Slow; a brute-force cross-check. */
void msda_oracle_encode_e4m3_exhaustive(const float* x, int64_t n, uint8_t* codes)
{
    for (int64_t i = 0; i < n; ++i) {
        double v = (double)x[i];
        unsigned sign = 0;
        if (signbit(v)) { sign = 0x80; v = -v; }
        if (v > 448.0) v = 448.0;
        unsigned best = 0;
        double bestd = INFINITY;
        for (unsigned q = 0; q < 127; ++q) {
            const int e = (q >> 3) & 15, m = q & 7;
            const double r = (e == 0) ? ldexp((double)m, -9) : ldexp(8.0 + (double)m, e - 10);
            const double d = fabs(r - v);
            if (d < bestd || (d == bestd && (q & 1) == 0)) { bestd = d; best = q; }
        }
        codes[i] = (uint8_t)(sign | best);
    }
}
