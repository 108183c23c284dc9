/*
 * Driver for the sanitizer build of the FP64 oracle (test infrastructure):
 * compiled together with oracle/msda_oracle.c under AddressSanitizer and
 * UndefinedBehaviorSanitizer by tests/test_oracle_sanitizers.py, it runs the
 * oracle's entry points on exactly sized heap buffers over the edge cases of
 * the operator -- samples fully and partly outside their level, 1x1 levels,
 * locations on the -1 and W edges, NaN and huge locations, overlapping
 * regions (the serial grad_feat path), one camera / level / keypoint -- and
 * over every FP8 code, so any read or write outside a buffer, or undefined
 * arithmetic, stops the run with a report. Prints "ok" at the end.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

void msda_oracle_forward(int B, int N, int L, int A, int P, int C, int G, int64_t R,
                         const double* feat, const int32_t* spatial_shapes,
                         const int32_t* level_start_index, const double* sampling_loc,
                         const double* weights, double* out, int nthreads);
void msda_oracle_backward(int B, int N, int L, int A, int P, int C, int G, int64_t R,
                          const double* feat, const int32_t* spatial_shapes,
                          const int32_t* level_start_index, const double* sampling_loc,
                          const double* weights, const double* grad_out, double* grad_feat,
                          double* grad_loc, double* grad_w, int nthreads);
void msda_oracle_decode_e4m3(const uint8_t* codes, int64_t n, double* out);
void msda_oracle_encode_e4m3(const float* x, int64_t n, uint8_t* codes);
void msda_oracle_encode_e4m3_exhaustive(const float* x, int64_t n, uint8_t* codes);

static uint64_t rng_state = 0x9e3779b97f4a7c15ull;

/* splitmix64 -> uniform double in [0, 1) */
static double urand(void)
{
    uint64_t z = (rng_state += 0x9e3779b97f4a7c15ull);
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    z ^= z >> 31;
    return (double)(z >> 11) * (1.0 / 9007199254740992.0);
}

static double* dalloc(size_t n)
{
    double* p = (double*)malloc((n ? n : 1) * sizeof(double));
    if (!p) abort();
    for (size_t i = 0; i < n; ++i) p[i] = urand() * 2.0 - 1.0;
    return p;
}

/* One problem: N cameras sharing L level shapes, regions packed in order
 * (or all starting at row 0 when overlap != 0), locations drawn from
 * [lo, hi) with some set to special values. */
static void run_case(int B, int N, int L, int A, int P, int C, int G, const int* hw, double lo,
                     double hi, int overlap, int threads)
{
    int32_t* shapes = (int32_t*)malloc(sizeof(int32_t) * 2 * N * L);
    int32_t* starts = (int32_t*)malloc(sizeof(int32_t) * N * L);
    int64_t R = 0;
    for (int n = 0; n < N; ++n)
        for (int l = 0; l < L; ++l) {
            shapes[2 * (n * L + l)] = hw[2 * l];
            shapes[2 * (n * L + l) + 1] = hw[2 * l + 1];
            const int64_t sz = (int64_t)hw[2 * l] * hw[2 * l + 1];
            if (overlap) {
                starts[n * L + l] = 0;
                if (sz > R) R = sz;
            } else {
                starts[n * L + l] = (int32_t)R;
                R += sz;
            }
        }
    const size_t nloc = (size_t)B * A * P * N * 2, nw = (size_t)B * A * P * N * L * G;
    double* feat = dalloc((size_t)B * R * C);
    double* loc = dalloc(nloc);
    for (size_t i = 0; i < nloc; ++i) loc[i] = lo + (hi - lo) * urand();
    /* special locations: the edges of a level of width W_0 (x = -1, x = W - 1,
     * x = W), NaN, huge values */
    const double W0 = hw[1];
    const double special[] = {-0.5 / W0, (W0 - 0.5) / W0, (W0 + 0.5) / W0, 0.0, 1.0, NAN,
                              1e30, -1e30, INFINITY, -INFINITY, 0.5 / W0, 1.0 - 1e-12};
    const size_t nspecial = sizeof(special) / sizeof(special[0]);
    for (size_t i = 0; i < nloc && i < 4 * nspecial; i += 2) loc[i] = special[(i / 2) % nspecial];
    double* w = dalloc(nw);
    double* go = dalloc((size_t)B * A * C);
    double* out = dalloc((size_t)B * A * C);
    double* gf = dalloc((size_t)B * R * C);
    double* gl = dalloc(nloc);
    double* gw = dalloc(nw);
    msda_oracle_forward(B, N, L, A, P, C, G, R, feat, shapes, starts, loc, w, out, threads);
    msda_oracle_backward(B, N, L, A, P, C, G, R, feat, shapes, starts, loc, w, go, gf, gl, gw,
                         threads);
    /* partial requests */
    msda_oracle_backward(B, N, L, A, P, C, G, R, feat, shapes, starts, loc, w, go, NULL, gl, NULL,
                         threads);
    msda_oracle_backward(B, N, L, A, P, C, G, R, feat, shapes, starts, loc, w, go, gf, NULL, NULL,
                         threads);
    /* outputs are finite (NaN / huge locations are skipped samples) */
    for (size_t i = 0; i < (size_t)B * A * C; ++i)
        if (!isfinite(out[i])) { fprintf(stderr, "non-finite out\n"); abort(); }
    free(shapes); free(starts); free(feat); free(loc); free(w); free(go); free(out);
    free(gf); free(gl); free(gw);
}

int main(void)
{
    const int pyr[] = {8, 14, 4, 7, 2, 4, 1, 2};
    const int ragged[] = {11, 13, 6, 7, 3, 3};
    const int ones[] = {1, 1, 1, 1};
    const int wide[] = {1, 9, 9, 1};
    run_case(1, 2, 4, 5, 3, 16, 4, pyr, -0.05, 1.05, 0, 1);
    run_case(2, 3, 3, 4, 2, 8, 2, ragged, -1.5, 2.5, 0, 4);      /* many fully outside */
    run_case(1, 2, 2, 3, 2, 4, 1, ones, -0.6, 1.6, 0, 2);        /* 1x1 levels */
    run_case(2, 2, 2, 3, 2, 6, 3, wide, -0.2, 1.2, 0, 3);        /* 1x9 and 9x1 */
    run_case(1, 3, 3, 4, 2, 8, 4, ragged, -0.1, 1.1, 1, 4);      /* overlapping regions */
    run_case(1, 1, 1, 1, 1, 1, 1, ones, 0.0, 1.0, 0, 1);         /* every size 1 */
    run_case(1, 2, 1, 0, 2, 4, 2, ragged, 0.0, 1.0, 0, 2);       /* no anchors */

    /* every FP8 code, and the encoders over a sweep with ties and clamps */
    uint8_t codes[256];
    double dec[256];
    for (int i = 0; i < 256; ++i) codes[i] = (uint8_t)i;
    msda_oracle_decode_e4m3(codes, 256, dec);
    enum { NX = 4096 };
    float* x = (float*)malloc(sizeof(float) * NX);
    uint8_t* c1 = (uint8_t*)malloc(NX);
    uint8_t* c2 = (uint8_t*)malloc(NX);
    for (int i = 0; i < NX; ++i) x[i] = (float)((urand() * 2.0 - 1.0) * 600.0 * urand());
    x[0] = 0.0f; x[1] = -0.0f; x[2] = 448.0f; x[3] = 464.0f; x[4] = 1e30f; x[5] = -INFINITY;
    x[6] = 0x1p-10f; x[7] = 0x1p-9f; x[8] = 0x1.8p-9f; x[9] = 1.0e-40f;
    msda_oracle_encode_e4m3(x, NX, c1);
    msda_oracle_encode_e4m3_exhaustive(x, NX, c2);
    for (int i = 0; i < NX; ++i)
        if (c1[i] != c2[i]) { fprintf(stderr, "encoders disagree at %d\n", i); abort(); }
    free(x); free(c1); free(c2);
    printf("ok\n");
    return 0;
}
