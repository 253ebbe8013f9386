/*
 * CPU oracle for asymmetric bidirectional optical flow stitching
 * (Meng & Liu, "High-quality Panorama Stitching based on Asymmetric
 * Bidirectional Optical Flow", arXiv 2006.01201).
 *
 * TEST INFRASTRUCTURE ONLY. This file is the plain, slow reference that the
 * GPU path is checked against. Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load it. It shares no code, header,
 * table or constant generator with the GPU library.
 *
 * Precision: integer stages in int32, floating-point stages in double.
 * Loops are written in the order the method states them; OpenMP only
 * splits the outer row loop (every row is independent).
 *
 * What the paper fixes and what is a reading of it:
 *   - Section III.C.1: two dense flows per overlap strip, FlowRtoL (of
 *     OverlappedR relative to OverlappedL) and FlowLtoR, computed by a
 *     coarse-to-fine pyramid method whose details the paper leaves out.
 *     The coarse-to-fine method below (luma, binomial pyramid, integer
 *     patch-cost search, Jacobi propagation, median smoothing, level-0
 *     Lucas-Kanade refinement) is the reading adopted for it; every
 *     constant of it is a parameter.
 *   - Flow convention: Ref(p) ~ Tgt(p + u(p)). FlowRtoL has Ref = R,
 *     Tgt = L, so R(p) ~ L(p + FlowRtoL(p)); this is the sense in which
 *     Code 1 displaces L by FlowRtoL.
 *   - eq. (1): the global blending coefficient; for a rectangular strip the
 *     minimum distances to Area1 / Area2 are x+1 and W-x (pixel centres).
 *   - Code 1: per-pixel asymmetric warp and softmax composite.
 *   - Canvas (eq. (1) and Code 1 with coverage masks of any shape): Area1
 *     / Area2 / Area3 come from the two masks, Lmin / Rmin are brute-force
 *     distances between pixel centres, and OverlappedL / OverlappedR are the
 *     crops of the bounding box of Area3.
 *   - The energy and its gradients (photometric Charbonnier + TV) are not
 *     in the paper; they define the flow-refinement extension.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

static inline int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Threads used by the parallel loops from now on (timing runs). */
void orc_set_num_threads(int n)
{
#ifdef _OPENMP
    omp_set_num_threads(n > 0 ? n : 1);
#else
    (void)n;
#endif
}

/* ------------------------------------------------------------------ */
/* Flow, step 1: intensity image. The paper runs its flow on image
 * intensity (Section III.C.1); the integer luma weights are a reading. */
void orc_luma(const uint8_t *rgb, int H, int W, long pitch, uint8_t *Y)
{
#pragma omp parallel for
    for (int y = 0; y < H; y++)
        for (int x = 0; x < W; x++) {
            const uint8_t *px = rgb + (long)y * pitch + 3L * x;
            int v = 77 * px[0] + 150 * px[1] + 29 * px[2] + 128;
            Y[(long)y * W + x] = (uint8_t)(v >> 8);
        }
}

/* Flow, step 1b: exposure compensation of R's intensity. The paper's
 * pre-processing corrects chromaticity between cameras (Section III.B);
 * the flow stage removes a residual global gain by scaling R's intensity
 * with the ratio of the two strips' intensity sums, in 16-bit fixed point:
 * a = floor(2^16 sum(YL) / sum(YR)), YR' = min(255, (YR a + 2^15) >> 16).
 * (An all-zero YR is left as it is.) */
void orc_gain_comp(const uint8_t *yl, uint8_t *yr, long n)
{
    long long sl = 0, sr = 0;
    for (long i = 0; i < n; i++) {
        sl += yl[i];
        sr += yr[i];
    }
    if (sr == 0) return;
    long long a = (sl << 16) / sr;
    for (long i = 0; i < n; i++) {
        long long v = ((long long)yr[i] * a + (1LL << 15)) >> 16;
        yr[i] = (uint8_t)(v > 255 ? 255 : v);
    }
}

/* Flow, step 2: one pyramid reduction. 5x5 binomial filter (weights
 * 1 4 6 4 1 in each direction, total 256), sampled at even positions,
 * borders clamped, one rounding. Output is ceil(H/2) x ceil(W/2). */
void orc_pyr_down(const uint8_t *src, int H, int W, uint8_t *dst)
{
    static const int w[5] = {1, 4, 6, 4, 1};
    int H2 = (H + 1) / 2, W2 = (W + 1) / 2;
#pragma omp parallel for
    for (int y = 0; y < H2; y++)
        for (int x = 0; x < W2; x++) {
            int s = 0;
            for (int j = 0; j < 5; j++)
                for (int i = 0; i < 5; i++) {
                    int sy = clampi(2 * y + j - 2, 0, H - 1);
                    int sx = clampi(2 * x + i - 2, 0, W - 1);
                    s += w[j] * w[i] * src[(long)sy * W + sx];
                }
            dst[(long)y * W2 + x] = (uint8_t)((s + 128) >> 8);
        }
}

/* Patch cost: sum over the (2P+1)^2 patch of |Ref - Tgt displaced by d|,
 * each coordinate clamped to the image on its own. */
static int patch_cost(const uint8_t *ref, const uint8_t *tgt, int H, int W,
                      int x, int y, int dx, int dy, int P)
{
    int c = 0;
    for (int j = -P; j <= P; j++)
        for (int i = -P; i <= P; i++) {
            int ry = clampi(y + j, 0, H - 1), rx = clampi(x + i, 0, W - 1);
            int ty = clampi(y + j + dy, 0, H - 1), tx = clampi(x + i + dx, 0, W - 1);
            c += abs((int)ref[(long)ry * W + rx] - (int)tgt[(long)ty * W + tx]);
        }
    return c;
}

/* Flow, step 3: centres of the next finer level from the coarser flow:
 * nearest-neighbour upsampling, values doubled. */
void orc_upsample(const int32_t *Dc, int Hc, int Wc, int H, int W, int32_t *centre)
{
#pragma omp parallel for
    for (int y = 0; y < H; y++)
        for (int x = 0; x < W; x++) {
            int cy = clampi(y / 2, 0, Hc - 1), cx = clampi(x / 2, 0, Wc - 1);
            centre[2 * ((long)y * W + x) + 0] = 2 * Dc[2 * ((long)cy * Wc + cx) + 0];
            centre[2 * ((long)y * W + x) + 1] = 2 * Dc[2 * ((long)cy * Wc + cx) + 1];
        }
}

/* Flow, step 4: integer patch-cost search around the centre. Candidates
 * d = c + (i, j), row offset j outer and column offset i inner, both from
 * -R to R. The winner is the lexicographic minimum of
 * (cost, |i| + |j|, enumeration index). centre == NULL means c = 0. */
void orc_search(const uint8_t *ref, const uint8_t *tgt, int H, int W,
                const int32_t *centre, int P, int R, int32_t *D, int32_t *cost)
{
#pragma omp parallel for
    for (int y = 0; y < H; y++)
        for (int x = 0; x < W; x++) {
            long p = (long)y * W + x;
            int cx = centre ? centre[2 * p] : 0, cy = centre ? centre[2 * p + 1] : 0;
            int best_c = 0, best_l1 = 0, best_idx = -1, bx = 0, by = 0;
            int idx = 0;
            for (int j = -R; j <= R; j++)
                for (int i = -R; i <= R; i++, idx++) {
                    int c = patch_cost(ref, tgt, H, W, x, y, cx + i, cy + j, P);
                    int l1 = abs(i) + abs(j);
                    int better = best_idx < 0 || c < best_c || (c == best_c && l1 < best_l1) ||
                                 (c == best_c && l1 == best_l1 && idx < best_idx);
                    if (better) {
                        best_c = c;
                        best_l1 = l1;
                        best_idx = idx;
                        bx = cx + i;
                        by = cy + j;
                    }
                }
            D[2 * p] = bx;
            D[2 * p + 1] = by;
            if (cost) cost[p] = best_c;
        }
}

/* Flow, step 5: T Jacobi propagation steps. Each pixel takes, from the
 * previous iterate only, the candidate with the lowest patch cost among
 * itself, left, right, up and down (neighbours outside the image are
 * skipped); on equal cost the earlier candidate in that order wins. */
void orc_propagate(const uint8_t *ref, const uint8_t *tgt, int H, int W, int P, int T,
                   const int32_t *Din, int32_t *Dout)
{
    long n = (long)H * W;
    int32_t *prev = (int32_t *)malloc(sizeof(int32_t) * 2 * n);
    memcpy(prev, Din, sizeof(int32_t) * 2 * n);
    memcpy(Dout, Din, sizeof(int32_t) * 2 * n);
    static const int nb[5][2] = {{0, 0}, {-1, 0}, {1, 0}, {0, -1}, {0, 1}};
    for (int t = 0; t < T; t++) {
#pragma omp parallel for
        for (int y = 0; y < H; y++)
            for (int x = 0; x < W; x++) {
                long p = (long)y * W + x;
                int best = -1, bx = 0, by = 0;
                for (int k = 0; k < 5; k++) {
                    int qx = x + nb[k][0], qy = y + nb[k][1];
                    if (qx < 0 || qx >= W || qy < 0 || qy >= H) continue;
                    long q = (long)qy * W + qx;
                    int dx = prev[2 * q], dy = prev[2 * q + 1];
                    int c = patch_cost(ref, tgt, H, W, x, y, dx, dy, P);
                    if (best < 0 || c < best) {
                        best = c;
                        bx = dx;
                        by = dy;
                    }
                }
                Dout[2 * p] = bx;
                Dout[2 * p + 1] = by;
            }
        memcpy(prev, Dout, sizeof(int32_t) * 2 * n);
    }
    free(prev);
}

static int cmp_int(const void *a, const void *b)
{
    int x = *(const int *)a, y = *(const int *)b;
    return (x > y) - (x < y);
}

/* Flow, step 6: component-wise (2M+1)^2 median with clamped indices. */
void orc_median(const int32_t *D, int H, int W, int M, int32_t *out)
{
    int k = (2 * M + 1) * (2 * M + 1);
#pragma omp parallel for
    for (int y = 0; y < H; y++) {
        int vals[121];
        for (int x = 0; x < W; x++)
            for (int comp = 0; comp < 2; comp++) {
                int n = 0;
                for (int j = -M; j <= M; j++)
                    for (int i = -M; i <= M; i++) {
                        int sy = clampi(y + j, 0, H - 1), sx = clampi(x + i, 0, W - 1);
                        vals[n++] = D[2 * ((long)sy * W + sx) + comp];
                    }
                qsort(vals, (size_t)n, sizeof(int), cmp_int);
                out[2 * ((long)y * W + x) + comp] = vals[k / 2];
            }
    }
}

/* Level sizes: level 0 is H x W, each next level ceil(/2). */
void orc_level_sizes(int H, int W, int N, int32_t *hs, int32_t *ws)
{
    for (int k = 0; k < N; k++) {
        hs[k] = H;
        ws[k] = W;
        H = (H + 1) / 2;
        W = (W + 1) / 2;
    }
}

/* The integer coarse-to-fine chain for one direction, from the level-0
 * intensity images. Writes, for every level k (concatenated, level 0
 * first, 2 ints per pixel), the raw search result and the final flow of
 * that level (after propagation and median). */
void orc_flow_int(const uint8_t *yref, const uint8_t *ytgt, int H, int W, int N,
                  int P, int R, int Rc, int T, int M,
                  int32_t *search_all, int32_t *final_all)
{
    int32_t hs[32], ws[32];
    long off[33] = {0};
    orc_level_sizes(H, W, N, hs, ws);
    off[0] = 0;
    for (int k = 0; k < N; k++) off[k + 1] = off[k] + (long)hs[k] * ws[k];

    uint8_t **pr = (uint8_t **)calloc(N, sizeof(uint8_t *));
    uint8_t **pt = (uint8_t **)calloc(N, sizeof(uint8_t *));
    pr[0] = (uint8_t *)malloc(off[1]);
    pt[0] = (uint8_t *)malloc(off[1]);
    memcpy(pr[0], yref, off[1]);
    memcpy(pt[0], ytgt, off[1]);
    for (int k = 1; k < N; k++) {
        pr[k] = (uint8_t *)malloc(off[k + 1] - off[k]);
        pt[k] = (uint8_t *)malloc(off[k + 1] - off[k]);
        orc_pyr_down(pr[k - 1], hs[k - 1], ws[k - 1], pr[k]);
        orc_pyr_down(pt[k - 1], hs[k - 1], ws[k - 1], pt[k]);
    }
    int32_t *centre = (int32_t *)malloc(sizeof(int32_t) * 2 * off[1]);
    int32_t *tmp = (int32_t *)malloc(sizeof(int32_t) * 2 * off[1]);
    for (int k = N - 1; k >= 0; k--) {
        int32_t *ds = search_all + 2 * off[k];
        int32_t *df = final_all + 2 * off[k];
        const int32_t *c = NULL;
        if (k < N - 1) {
            orc_upsample(final_all + 2 * off[k + 1], hs[k + 1], ws[k + 1], hs[k], ws[k], centre);
            c = centre;
        }
        orc_search(pr[k], pt[k], hs[k], ws[k], c, P, k == N - 1 ? Rc : R, ds, NULL);
        orc_propagate(pr[k], pt[k], hs[k], ws[k], P, T, ds, tmp);
        if (M > 0)
            orc_median(tmp, hs[k], ws[k], M, df);
        else
            memcpy(df, tmp, sizeof(int32_t) * 2 * (off[k + 1] - off[k]));
    }
    for (int k = 0; k < N; k++) {
        free(pr[k]);
        free(pt[k]);
    }
    free(pr);
    free(pt);
    free(centre);
    free(tmp);
}

/* Bilinear sample of a single-channel image at (x0 + fx, y0 + fy), with
 * integer cell corner (x0, y0), fractions in [0, 1), indices clamped. */
static double bilin1(const uint8_t *img, int H, int W, int x0, int y0, double fx, double fy)
{
    int xa = clampi(x0, 0, W - 1), xb = clampi(x0 + 1, 0, W - 1);
    int ya = clampi(y0, 0, H - 1), yb = clampi(y0 + 1, 0, H - 1);
    double v00 = img[(long)ya * W + xa], v01 = img[(long)ya * W + xb];
    double v10 = img[(long)yb * W + xa], v11 = img[(long)yb * W + xb];
    return (1 - fy) * ((1 - fx) * v00 + fx * v01) + fy * ((1 - fx) * v10 + fx * v11);
}

/* Flow, step 7: sub-pixel refinement at level 0 (Lucas-Kanade,
 * Gauss-Newton). A = Ref intensity, B = Tgt intensity. Central-difference
 * gradient of A; normal matrix summed over the (2Plk+1)^2 window plus
 * eps * I; Klk iterations from the integer flow; each component clamped to
 * within 1 px of the integer flow. */
void orc_refine(const uint8_t *A, const uint8_t *B, int H, int W, const int32_t *D0,
                int Plk, int Klk, double eps, double *u_out)
{
#pragma omp parallel for
    for (int y = 0; y < H; y++)
        for (int x = 0; x < W; x++) {
            long p = (long)y * W + x;
            double hxx = eps, hxy = 0, hyy = eps;
            for (int j = -Plk; j <= Plk; j++)
                for (int i = -Plk; i <= Plk; i++) {
                    int qy = clampi(y + j, 0, H - 1), qx = clampi(x + i, 0, W - 1);
                    double gx = 0.5 * ((double)A[(long)qy * W + clampi(qx + 1, 0, W - 1)] -
                                       (double)A[(long)qy * W + clampi(qx - 1, 0, W - 1)]);
                    double gy = 0.5 * ((double)A[(long)clampi(qy + 1, 0, H - 1) * W + qx] -
                                       (double)A[(long)clampi(qy - 1, 0, H - 1) * W + qx]);
                    hxx += gx * gx;
                    hxy += gx * gy;
                    hyy += gy * gy;
                }
            double det = hxx * hyy - hxy * hxy;
            double ux = D0[2 * p], uy = D0[2 * p + 1];
            double lox = ux - 1, hix = ux + 1, loy = uy - 1, hiy = uy + 1;
            for (int it = 0; it < Klk; it++) {
                double fux = floor(ux), fuy = floor(uy);
                double fx = ux - fux, fy = uy - fuy;
                double bx = 0, by = 0;
                for (int j = -Plk; j <= Plk; j++)
                    for (int i = -Plk; i <= Plk; i++) {
                        int qy = clampi(y + j, 0, H - 1), qx = clampi(x + i, 0, W - 1);
                        double gx = 0.5 * ((double)A[(long)qy * W + clampi(qx + 1, 0, W - 1)] -
                                           (double)A[(long)qy * W + clampi(qx - 1, 0, W - 1)]);
                        double gy = 0.5 * ((double)A[(long)clampi(qy + 1, 0, H - 1) * W + qx] -
                                           (double)A[(long)clampi(qy - 1, 0, H - 1) * W + qx]);
                        double e = bilin1(B, H, W, qx + (int)fux, qy + (int)fuy, fx, fy) -
                                   (double)A[(long)qy * W + qx];
                        bx += gx * e;
                        by += gy * e;
                    }
                double dx = -(hyy * bx - hxy * by) / det;
                double dy = -(hxx * by - hxy * bx) / det;
                ux += dx;
                uy += dy;
                ux = ux < lox ? lox : (ux > hix ? hix : ux);
                uy = uy < loy ? loy : (uy > hiy ? hiy : uy);
            }
            u_out[2 * p] = ux;
            u_out[2 * p + 1] = uy;
        }
}

/* ------------------------------------------------------------------ */
/* Classic coarse-to-fine Lucas-Kanade (the "LK pyramid" of III.C.1, as an
 * alternative to the integer search): float flows at every level. */

/* One level: A = Ref, B = Tgt intensity (H x W). The flow of every pixel
 * starts at seed (H x W x 2; NULL = 0) and takes K Gauss-Newton steps
 * u <- u - (sum g g^T + eps I)^-1 sum g (B~(q + u) - A(q)) over the
 * (2P+1)^2 window, g the central-difference gradient of A, B~ bilinear
 * with clamped indices; no clamp on u. */
void orc_lk_level(const uint8_t *A, const uint8_t *B, int H, int W, const double *seed, int P, int K, double eps,
                  double *u_out)
{
#pragma omp parallel for
    for (int y = 0; y < H; y++)
        for (int x = 0; x < W; x++) {
            long p = (long)y * W + x;
            double hxx = eps, hxy = 0, hyy = eps;
            for (int j = -P; j <= P; j++)
                for (int i = -P; i <= P; i++) {
                    int qy = clampi(y + j, 0, H - 1), qx = clampi(x + i, 0, W - 1);
                    double gx = 0.5 * ((double)A[(long)qy * W + clampi(qx + 1, 0, W - 1)] -
                                       (double)A[(long)qy * W + clampi(qx - 1, 0, W - 1)]);
                    double gy = 0.5 * ((double)A[(long)clampi(qy + 1, 0, H - 1) * W + qx] -
                                       (double)A[(long)clampi(qy - 1, 0, H - 1) * W + qx]);
                    hxx += gx * gx;
                    hxy += gx * gy;
                    hyy += gy * gy;
                }
            double det = hxx * hyy - hxy * hxy;
            double ux = seed ? seed[2 * p] : 0.0, uy = seed ? seed[2 * p + 1] : 0.0;
            for (int it = 0; it < K; it++) {
                double fux = floor(ux), fuy = floor(uy);
                double fx = ux - fux, fy = uy - fuy;
                double bx = 0, by = 0;
                for (int j = -P; j <= P; j++)
                    for (int i = -P; i <= P; i++) {
                        int qy = clampi(y + j, 0, H - 1), qx = clampi(x + i, 0, W - 1);
                        double gx = 0.5 * ((double)A[(long)qy * W + clampi(qx + 1, 0, W - 1)] -
                                           (double)A[(long)qy * W + clampi(qx - 1, 0, W - 1)]);
                        double gy = 0.5 * ((double)A[(long)clampi(qy + 1, 0, H - 1) * W + qx] -
                                           (double)A[(long)clampi(qy - 1, 0, H - 1) * W + qx]);
                        double e = bilin1(B, H, W, qx + (int)fux, qy + (int)fuy, fx, fy) -
                                   (double)A[(long)qy * W + qx];
                        bx += gx * e;
                        by += gy * e;
                    }
                ux -= (hyy * bx - hxy * by) / det;
                uy -= (hxx * by - hxy * bx) / det;
            }
            u_out[2 * p] = ux;
            u_out[2 * p + 1] = uy;
        }
}

/* One direction over the pyramid: level N-1 from 0, every finer level k
 * from 2 u_{k+1}(floor(x/2), floor(y/2)) (clamped to the coarser size).
 * Writes every level's flow (concatenated, level 0 first, 2 doubles per
 * pixel) to flow_all. */
void orc_flow_lk(const uint8_t *yref, const uint8_t *ytgt, int H, int W, int N, int P, int K, double eps,
                 double *flow_all)
{
    int32_t hs[32], ws[32];
    long off[33] = {0};
    orc_level_sizes(H, W, N, hs, ws);
    for (int k = 0; k < N; k++) off[k + 1] = off[k] + (long)hs[k] * ws[k];
    uint8_t **pr = (uint8_t **)calloc(N, sizeof(uint8_t *));
    uint8_t **pt = (uint8_t **)calloc(N, sizeof(uint8_t *));
    pr[0] = (uint8_t *)malloc(off[1]);
    pt[0] = (uint8_t *)malloc(off[1]);
    memcpy(pr[0], yref, off[1]);
    memcpy(pt[0], ytgt, off[1]);
    for (int k = 1; k < N; k++) {
        pr[k] = (uint8_t *)malloc(off[k + 1] - off[k]);
        pt[k] = (uint8_t *)malloc(off[k + 1] - off[k]);
        orc_pyr_down(pr[k - 1], hs[k - 1], ws[k - 1], pr[k]);
        orc_pyr_down(pt[k - 1], hs[k - 1], ws[k - 1], pt[k]);
    }
    double *seed = (double *)malloc(sizeof(double) * 2 * off[1]);
    for (int k = N - 1; k >= 0; k--) {
        const double *sd = NULL;
        if (k < N - 1) {
            const double *c = flow_all + 2 * off[k + 1];
            for (int y = 0; y < hs[k]; y++)
                for (int x = 0; x < ws[k]; x++) {
                    long q = (long)clampi(y / 2, 0, hs[k + 1] - 1) * ws[k + 1] + clampi(x / 2, 0, ws[k + 1] - 1);
                    seed[2 * ((long)y * ws[k] + x)] = 2.0 * c[2 * q];
                    seed[2 * ((long)y * ws[k] + x) + 1] = 2.0 * c[2 * q + 1];
                }
            sd = seed;
        }
        orc_lk_level(pr[k], pt[k], hs[k], ws[k], sd, P, K, eps, flow_all + 2 * off[k]);
    }
    for (int k = 0; k < N; k++) {
        free(pr[k]);
        free(pt[k]);
    }
    free(pr);
    free(pt);
    free(seed);
}

/* Both flows of one strip with the classic method (luma and exposure step
 * as in the integer chain). flow_all_lr / flow_all_rl: every level, as in
 * orc_flow_lk (level 0 first). */
void orc_flow_lk_bidirectional(const uint8_t *L, const uint8_t *R, int H, int W, long pitchL, long pitchR, int N,
                               int P, int K, double eps, int gain, double *flow_all_lr, double *flow_all_rl)
{
    long n = (long)H * W;
    uint8_t *yl = (uint8_t *)malloc(n), *yr = (uint8_t *)malloc(n);
    orc_luma(L, H, W, pitchL, yl);
    orc_luma(R, H, W, pitchR, yr);
    if (gain) orc_gain_comp(yl, yr, n);
    orc_flow_lk(yl, yr, H, W, N, P, K, eps, flow_all_lr);
    orc_flow_lk(yr, yl, H, W, N, P, K, eps, flow_all_rl);
    free(yl);
    free(yr);
}

/* Both flows of one strip (Section III.C.1). FlowLtoR: Ref = L, Tgt = R.
 * FlowRtoL: Ref = R, Tgt = L; with `gain`, R's intensity is compensated
 * first (step 1b) and both directions use it. Optional integer outputs: per-level search
 * results and final flows for each direction (layout of orc_flow_int). */
void orc_flow_bidirectional(const uint8_t *L, const uint8_t *R, int H, int W, long pitchL, long pitchR,
                            int N, int P, int Rs, int Rc, int T, int M, int Plk, int Klk, double eps, int gain,
                            double *flow_lr, double *flow_rl,
                            int32_t *search_lr, int32_t *final_lr, int32_t *search_rl, int32_t *final_rl)
{
    long n = (long)H * W, tot = 0;
    int32_t hs[32], ws[32];
    orc_level_sizes(H, W, N, hs, ws);
    for (int k = 0; k < N; k++) tot += (long)hs[k] * ws[k];
    uint8_t *yl = (uint8_t *)malloc(n), *yr = (uint8_t *)malloc(n);
    orc_luma(L, H, W, pitchL, yl);
    orc_luma(R, H, W, pitchR, yr);
    if (gain) orc_gain_comp(yl, yr, n);
    int32_t *s1 = search_lr ? search_lr : (int32_t *)malloc(sizeof(int32_t) * 2 * tot);
    int32_t *f1 = final_lr ? final_lr : (int32_t *)malloc(sizeof(int32_t) * 2 * tot);
    int32_t *s2 = search_rl ? search_rl : (int32_t *)malloc(sizeof(int32_t) * 2 * tot);
    int32_t *f2 = final_rl ? final_rl : (int32_t *)malloc(sizeof(int32_t) * 2 * tot);
    orc_flow_int(yl, yr, H, W, N, P, Rs, Rc, T, M, s1, f1);
    orc_flow_int(yr, yl, H, W, N, P, Rs, Rc, T, M, s2, f2);
    orc_refine(yl, yr, H, W, f1, Plk, Klk, eps, flow_lr);
    orc_refine(yr, yl, H, W, f2, Plk, Klk, eps, flow_rl);
    if (!search_lr) free(s1);
    if (!final_lr) free(f1);
    if (!search_rl) free(s2);
    if (!final_rl) free(f2);
    free(yl);
    free(yr);
}

/* ------------------------------------------------------------------ */
/* Blend */

/* eq. (1) for a rectangular strip: Lmin = distance to the nearest Area1
 * pixel centre, Rmin = to the nearest Area2 pixel centre. axis 0: Area1
 * left of the strip, Area2 right; axis 1: Area1 above, Area2 below. */
double orc_blend_coef(int x, int y, int H, int W, int axis)
{
    double lmin = axis == 0 ? x + 1.0 : y + 1.0;
    double rmin = axis == 0 ? (double)(W - x) : (double)(H - y);
    return lmin / (lmin + rmin);
}

static double finite_or_zero(double v) { return isfinite(v) ? v : 0.0; }

/* Bilinear RGB sample at (x0 + fx, y0 + fy) of a double H x W x 3 image. */
static void bilin3(const double *img, int H, int W, int x0, int y0, double fx, double fy, double out[3])
{
    int xa = clampi(x0, 0, W - 1), xb = clampi(x0 + 1, 0, W - 1);
    int ya = clampi(y0, 0, H - 1), yb = clampi(y0 + 1, 0, H - 1);
    for (int c = 0; c < 3; c++) {
        double v00 = img[3 * ((long)ya * W + xa) + c], v01 = img[3 * ((long)ya * W + xb) + c];
        double v10 = img[3 * ((long)yb * W + xa) + c], v11 = img[3 * ((long)yb * W + xb) + c];
        out[c] = (1 - fy) * ((1 - fx) * v00 + fx * v01) + fy * ((1 - fx) * v10 + fx * v11);
    }
}

/* Code 1 over one strip (all of it is Area3). Images are double H x W x 3.
 * blend == NULL uses eq. (1). mode 0 = softmax composite (Code 1),
 * mode 1 = linear weights (SoftmaxR = Blend) for tests. Writes the
 * unrounded composite F (double) and, if F8 != NULL, clamp(floor(F+0.5)). */
void orc_blend(const double *L, const double *R, const double *flow_lr, const double *flow_rl,
               const double *blend, int axis, int H, int W, double kS, double kF, int mode,
               double *F, uint8_t *F8)
{
    double S = axis == 0 ? (double)W : (double)H;
#pragma omp parallel for
    for (int y = 0; y < H; y++)
        for (int x = 0; x < W; x++) {
            long p = (long)y * W + x;
            double t = blend ? blend[p] : orc_blend_coef(x, y, H, W, axis);
            double blendL = 1.0 - t, blendR = t;
            double frx = finite_or_zero(flow_rl[2 * p]), fry = finite_or_zero(flow_rl[2 * p + 1]);
            double flx = finite_or_zero(flow_lr[2 * p]), fly = finite_or_zero(flow_lr[2 * p + 1]);
            /* L is sampled at p + FlowRtoL * (1 - BlendL), R at
             * p + FlowLtoR * (1 - BlendR); the integer part of the
             * displacement is split off before adding the pixel index */
            double ax = frx * (1.0 - blendL), ay = fry * (1.0 - blendL);
            double bx = flx * (1.0 - blendR), by = fly * (1.0 - blendR);
            double cl[3], cr[3];
            bilin3(L, H, W, x + (int)floor(ax), y + (int)floor(ay), ax - floor(ax), ay - floor(ay), cl);
            bilin3(R, H, W, x + (int)floor(bx), y + (int)floor(by), bx - floor(bx), by - floor(by), cr);
            double sL, sR;
            if (mode == 1) {
                sR = t;
                sL = 1.0 - t;
            } else {
                double magRL = sqrt(frx * frx + fry * fry) / S;
                double magLR = sqrt(flx * flx + fly * fly) / S;
                double zL = kS * blendL * (1.0 + kF * magRL);
                double zR = kS * blendR * (1.0 + kF * magLR);
                /* exp(zL) / (exp(zL) + exp(zR)) in a form that cannot overflow */
                sL = 1.0 / (1.0 + exp(zR - zL));
                sR = 1.0 - sL;
            }
            for (int c = 0; c < 3; c++) {
                double f = sL * cl[c] + sR * cr[c];
                F[3 * p + c] = f;
                if (F8) {
                    double r = floor(f + 0.5);
                    F8[3 * p + c] = (uint8_t)(r < 0 ? 0 : (r > 255 ? 255 : r));
                }
            }
        }
}

/* Gradient of the bilinear sample of a double H x W x 3 image with respect
 * to the sample position, per channel; the derivative at an integer
 * position is the right-hand one (the cell starting there). */
static void bilin3_grad(const double *img, int H, int W, int x0, int y0, double fx, double fy,
                        double dX[3], double dY[3])
{
    int xa = clampi(x0, 0, W - 1), xb = clampi(x0 + 1, 0, W - 1);
    int ya = clampi(y0, 0, H - 1), yb = clampi(y0 + 1, 0, H - 1);
    for (int c = 0; c < 3; c++) {
        double v00 = img[3 * ((long)ya * W + xa) + c], v01 = img[3 * ((long)ya * W + xb) + c];
        double v10 = img[3 * ((long)yb * W + xa) + c], v11 = img[3 * ((long)yb * W + xb) + c];
        dX[c] = (1 - fy) * (v01 - v00) + fy * (v11 - v10);
        dY[c] = (1 - fx) * (v10 - v00) + fx * (v11 - v01);
    }
}

/* Adds w * (bilinear weights) of the sample at (x0 + fx, y0 + fy) into the
 * gradient image g (H x W x 3), channel c, at the clamped corners. */
static void bilin_scatter(double *g, int H, int W, int x0, int y0, double fx, double fy, int c, double w)
{
    int xa = clampi(x0, 0, W - 1), xb = clampi(x0 + 1, 0, W - 1);
    int ya = clampi(y0, 0, H - 1), yb = clampi(y0 + 1, 0, H - 1);
    g[3 * ((long)ya * W + xa) + c] += w * (1 - fy) * (1 - fx);
    g[3 * ((long)ya * W + xb) + c] += w * (1 - fy) * fx;
    g[3 * ((long)yb * W + xa) + c] += w * fy * (1 - fx);
    g[3 * ((long)yb * W + xb) + c] += w * fy * fx;
}

/* ------------------------------------------------------------------ */
/* Flow-refinement energy (an extension; not in the paper):
 *   E(u) = sum_p sum_c rho(Tgt~_c(p + u(p)) - Ref_c(p))
 *        + lambda * sum_p sum_m sqrt((dx u_m)^2 + (dy u_m)^2 + eps^2),
 * rho(r) = sqrt(r^2 + eps^2), Tgt~ bilinear with clamped indices, forward
 * differences that are 0 at the last column / row. Images are double
 * H x W x 3, u is H x W x 2. Gradient outputs may be NULL; they are
 * overwritten (not accumulated). Returns E. */
double orc_energy(const double *Ref, const double *Tgt, const double *u, int H, int W,
                  double lambda, double eps, double *g_u, double *g_ref, double *g_tgt)
{
    long n = (long)H * W;
    if (g_u) memset(g_u, 0, sizeof(double) * 2 * n);
    if (g_ref) memset(g_ref, 0, sizeof(double) * 3 * n);
    if (g_tgt) memset(g_tgt, 0, sizeof(double) * 3 * n);
    double E = 0;
    for (int y = 0; y < H; y++)
        for (int x = 0; x < W; x++) {
            long p = (long)y * W + x;
            double ux = u[2 * p], uy = u[2 * p + 1];
            double fux = floor(ux), fuy = floor(uy);
            int x0 = x + (int)fux, y0 = y + (int)fuy;
            double fx = ux - fux, fy = uy - fuy;
            double v[3], dX[3], dY[3];
            bilin3(Tgt, H, W, x0, y0, fx, fy, v);
            bilin3_grad(Tgt, H, W, x0, y0, fx, fy, dX, dY);
            for (int c = 0; c < 3; c++) {
                double r = v[c] - Ref[3 * p + c];
                double rho = sqrt(r * r + eps * eps);
                double drho = r / rho;
                E += rho;
                if (g_u) {
                    g_u[2 * p] += drho * dX[c];
                    g_u[2 * p + 1] += drho * dY[c];
                }
                if (g_ref) g_ref[3 * p + c] = -drho;
                if (g_tgt) bilin_scatter(g_tgt, H, W, x0, y0, fx, fy, c, drho);
            }
            for (int m = 0; m < 2; m++) {
                double dx = x < W - 1 ? u[2 * (p + 1) + m] - u[2 * p + m] : 0.0;
                double dy = y < H - 1 ? u[2 * (p + W) + m] - u[2 * p + m] : 0.0;
                double s = sqrt(dx * dx + dy * dy + eps * eps);
                E += lambda * s;
                if (g_u) {
                    if (x < W - 1) {
                        g_u[2 * (p + 1) + m] += lambda * dx / s;
                        g_u[2 * p + m] -= lambda * dx / s;
                    }
                    if (y < H - 1) {
                        g_u[2 * (p + W) + m] += lambda * dy / s;
                        g_u[2 * p + m] -= lambda * dy / s;
                    }
                }
            }
        }
    return E;
}

/* Gradient descent on the energy above: steps times
 * u <- u - clip(eta * dE/du, -clip_px, clip_px), per component, with a
 * fixed step and no early stop. Optionally records E before each step and
 * after the last one (steps + 1 values). */
void orc_refine_gd(const double *Ref, const double *Tgt, double *u, int H, int W, int steps,
                   double eta, double lambda, double eps, double clip_px, double *E_hist)
{
    long n = (long)H * W;
    double *g = (double *)malloc(sizeof(double) * 2 * n);
    for (int s = 0; s < steps; s++) {
        double E = orc_energy(Ref, Tgt, u, H, W, lambda, eps, g, NULL, NULL);
        if (E_hist) E_hist[s] = E;
        for (long i = 0; i < 2 * n; i++) {
            double d = eta * g[i];
            d = d < -clip_px ? -clip_px : (d > clip_px ? clip_px : d);
            u[i] -= d;
        }
    }
    if (E_hist) E_hist[steps] = orc_energy(Ref, Tgt, u, H, W, lambda, eps, NULL, NULL, NULL);
    free(g);
}

/* Adjoint of Code 1 (chain rule through orc_blend's float composite).
 * g_F is H x W x 3. Outputs (overwritten, any may be NULL): gradients with
 * respect to both flows (H x W x 2) and both images (H x W x 3). The
 * derivative of |f| is f/|f| for f != 0 and 0 at 0; a non-finite flow
 * component is used as 0 and gets a zero gradient. */
void orc_blend_grad(const double *L, const double *R, const double *flow_lr, const double *flow_rl,
                    const double *blend, int axis, int H, int W, double kS, double kF, int mode,
                    const double *g_F, double *g_flow_lr, double *g_flow_rl, double *g_L, double *g_R)
{
    long n = (long)H * W;
    double S = axis == 0 ? (double)W : (double)H;
    if (g_flow_lr) memset(g_flow_lr, 0, sizeof(double) * 2 * n);
    if (g_flow_rl) memset(g_flow_rl, 0, sizeof(double) * 2 * n);
    if (g_L) memset(g_L, 0, sizeof(double) * 3 * n);
    if (g_R) memset(g_R, 0, sizeof(double) * 3 * n);
    for (int y = 0; y < H; y++)
        for (int x = 0; x < W; x++) {
            long p = (long)y * W + x;
            double t = blend ? blend[p] : orc_blend_coef(x, y, H, W, axis);
            int okrx = isfinite(flow_rl[2 * p]), okry = isfinite(flow_rl[2 * p + 1]);
            int oklx = isfinite(flow_lr[2 * p]), okly = isfinite(flow_lr[2 * p + 1]);
            double frx = okrx ? flow_rl[2 * p] : 0, fry = okry ? flow_rl[2 * p + 1] : 0;
            double flx = oklx ? flow_lr[2 * p] : 0, fly = okly ? flow_lr[2 * p + 1] : 0;
            double ax = frx * t, ay = fry * t, bx = flx * (1 - t), by = fly * (1 - t);
            int lx0 = x + (int)floor(ax), ly0 = y + (int)floor(ay);
            int rx0 = x + (int)floor(bx), ry0 = y + (int)floor(by);
            double lfx = ax - floor(ax), lfy = ay - floor(ay), rfx = bx - floor(bx), rfy = by - floor(by);
            double cl[3], cr[3], dLX[3], dLY[3], dRX[3], dRY[3];
            bilin3(L, H, W, lx0, ly0, lfx, lfy, cl);
            bilin3(R, H, W, rx0, ry0, rfx, rfy, cr);
            bilin3_grad(L, H, W, lx0, ly0, lfx, lfy, dLX, dLY);
            bilin3_grad(R, H, W, rx0, ry0, rfx, rfy, dRX, dRY);
            double sL, sR, nRL = sqrt(frx * frx + fry * fry), nLR = sqrt(flx * flx + fly * fly);
            if (mode == 1) {
                sR = t;
                sL = 1 - t;
            } else {
                double zL = kS * (1 - t) * (1 + kF * nRL / S);
                double zR = kS * t * (1 + kF * nLR / S);
                sL = 1.0 / (1.0 + exp(zR - zL));
                sR = 1.0 - sL;
            }
            /* dF/dColorL = SoftmaxL, dF/dColorR = SoftmaxR, dF/dSoftmaxL = ColorL - ColorR */
            double gs = 0, gLx = 0, gLy = 0, gRx = 0, gRy = 0;
            for (int c = 0; c < 3; c++) {
                double g = g_F[3 * p + c];
                gs += g * (cl[c] - cr[c]);
                gLx += g * sL * dLX[c];
                gLy += g * sL * dLY[c];
                gRx += g * sR * dRX[c];
                gRy += g * sR * dRY[c];
                if (g_L) bilin_scatter(g_L, H, W, lx0, ly0, lfx, lfy, c, g * sL);
                if (g_R) bilin_scatter(g_R, H, W, rx0, ry0, rfx, rfy, c, g * sR);
            }
            /* positions: dLx/dFlowRtoL.x = t, dRx/dFlowLtoR.x = 1 - t */
            double grl_x = t * gLx, grl_y = t * gLy, glr_x = (1 - t) * gRx, glr_y = (1 - t) * gRy;
            if (mode != 1) {
                /* SoftmaxL = sigma(zL - zR): d/dzL = sL*sR, d/dzR = -sL*sR */
                double dz = gs * sL * sR;
                if (nRL > 0) {
                    double k = dz * kS * (1 - t) * kF / S / nRL;
                    grl_x += k * frx;
                    grl_y += k * fry;
                }
                if (nLR > 0) {
                    double k = -dz * kS * t * kF / S / nLR;
                    glr_x += k * flx;
                    glr_y += k * fly;
                }
            }
            if (g_flow_rl) {
                g_flow_rl[2 * p] = okrx ? grl_x : 0;
                g_flow_rl[2 * p + 1] = okry ? grl_y : 0;
            }
            if (g_flow_lr) {
                g_flow_lr[2 * p] = oklx ? glr_x : 0;
                g_flow_lr[2 * p + 1] = okly ? glr_y : 0;
            }
        }
}

/* ------------------------------------------------------------------ */
/* Canvas: eq. (1) and Code 1 with coverage masks of any shape
 * (Section III.C: Area1 holds only L, Area2 only R, Area3 both). */

/* Area of canvas pixel (x, y) from the coverage masks (nonzero = the image
 * covers the pixel): 1 = only L, 2 = only R, 3 = both, 0 = neither. */
static int canvas_area(const uint8_t *mL, const uint8_t *mR, long pitch, int x, int y)
{
    int l = mL[(long)y * pitch + x] != 0, r = mR[(long)y * pitch + x] != 0;
    return l && r ? 3 : (l ? 1 : (r ? 2 : 0));
}

/* Column offset between canvas columns u and x: |u - x|, or, on a
 * periodic canvas (x wraps: column W - 1 neighbours column 0, as on a
 * 360-degree panorama), the shorter way round, min(|u - x|, W - |u - x|). */
static long long col_dist(int u, int x, int W, int periodic)
{
    long long d = u > x ? u - x : x - u;
    if (periodic && W - d < d) d = W - d;
    return d;
}

/* Squared Euclidean distance between the centre of (x, y) and the centre
 * of the nearest canvas pixel of area `a`, over every pixel of the canvas;
 * -1 when no pixel has that area. */
static long long nearest_d2(const uint8_t *mL, const uint8_t *mR, long pitch, int H, int W, int x, int y, int a,
                            int periodic)
{
    long long best = -1;
    for (int v = 0; v < H; v++)
        for (int u = 0; u < W; u++) {
            if (canvas_area(mL, mR, pitch, u, v) != a) continue;
            long long dx = col_dist(u, x, W, periodic);
            long long d = dx * dx + (long long)(v - y) * (v - y);
            if (best < 0 || d < best) best = d;
        }
    return best;
}

/* Squared distances from n canvas points to Area1 (d2_1) and Area2 (d2_2). */
void orc_canvas_dist2(const uint8_t *mL, const uint8_t *mR, long pitch, int H, int W, int periodic, long n,
                      const int32_t *xs, const int32_t *ys, long long *d2_1, long long *d2_2)
{
#pragma omp parallel for schedule(dynamic, 16)
    for (long i = 0; i < n; i++) {
        d2_1[i] = nearest_d2(mL, mR, pitch, H, W, xs[i], ys[i], 1, periodic);
        d2_2[i] = nearest_d2(mL, mR, pitch, H, W, xs[i], ys[i], 2, periodic);
    }
}

/* The same squared distances in two stages, for long lists of points on
 * large canvases: for every row v and column x, the distance along the
 * row to the nearest pixel of the area in that row (g_v(x), none if the
 * row has no such pixel; measured the shorter way round on a periodic
 * canvas); then the nearest pixel of the area to (x, y) is, for some row
 * v, the nearest one in that row, so
 * d^2(x, y) = min over v of (y - v)^2 + g_v(x)^2. */
static void row_distances(const uint8_t *mL, const uint8_t *mR, long pitch, int H, int W, int a, int periodic,
                          int32_t *g)
{
#pragma omp parallel for
    for (int v = 0; v < H; v++) {
        int32_t *row = g + (long)v * W;
        int first = -1, lastm = -1;  /* the row's first and last pixel of the area */
        for (int x = 0; x < W; x++)
            if (canvas_area(mL, mR, pitch, x, v) == a) {
                if (first < 0) first = x;
                lastm = x;
            }
        /* nearest member at or left of x; on a periodic canvas, with none,
         * the row's last member reached leftwards across column 0 */
        int last = -1;
        for (int x = 0; x < W; x++) {
            if (canvas_area(mL, mR, pitch, x, v) == a) last = x;
            row[x] = last >= 0 ? x - last : (periodic && lastm >= 0 ? x + W - lastm : -1);
        }
        /* nearest member at or right of x; with none, the first member
         * reached rightwards across column W - 1 */
        last = -1;
        for (int x = W - 1; x >= 0; x--) {
            if (canvas_area(mL, mR, pitch, x, v) == a) last = x;
            int d = last >= 0 ? last - x : (periodic && first >= 0 ? W - x + first : -1);
            if (d >= 0 && (row[x] < 0 || d < row[x])) row[x] = d;
        }
    }
}

void orc_canvas_dist2_rows(const uint8_t *mL, const uint8_t *mR, long pitch, int H, int W, int periodic, long n,
                           const int32_t *xs, const int32_t *ys, long long *d2_1, long long *d2_2)
{
    int32_t *g1 = (int32_t *)malloc(sizeof(int32_t) * (size_t)H * W);
    int32_t *g2 = (int32_t *)malloc(sizeof(int32_t) * (size_t)H * W);
    row_distances(mL, mR, pitch, H, W, 1, periodic, g1);
    row_distances(mL, mR, pitch, H, W, 2, periodic, g2);
#pragma omp parallel for schedule(dynamic, 64)
    for (long i = 0; i < n; i++) {
        const int x = xs[i], y = ys[i];
        long long b1 = -1, b2 = -1;
        for (int v = 0; v < H; v++) {
            const long long dy2 = (long long)(y - v) * (y - v);
            const int32_t a1 = g1[(long)v * W + x], a2 = g2[(long)v * W + x];
            if (a1 >= 0 && (b1 < 0 || dy2 + (long long)a1 * a1 < b1)) b1 = dy2 + (long long)a1 * a1;
            if (a2 >= 0 && (b2 < 0 || dy2 + (long long)a2 * a2 < b2)) b2 = dy2 + (long long)a2 * a2;
        }
        d2_1[i] = b1;
        d2_2[i] = b2;
    }
    free(g1);
    free(g2);
}

/* eq. (1) at n canvas points: 0 in Area1, 1 in Area2, 0.5 outside both
 * images, Lmin / (Lmin + Rmin) in Area3 with Lmin / Rmin the distances to
 * Area1 / Area2. An empty Area1 is infinitely far (Blend 1), an empty
 * Area2 likewise (Blend 0); with both empty Area3 takes 0.5. */
void orc_canvas_blend(const uint8_t *mL, const uint8_t *mR, long pitch, int H, int W, int periodic, long n,
                      const int32_t *xs, const int32_t *ys, double *out)
{
#pragma omp parallel for schedule(dynamic, 16)
    for (long i = 0; i < n; i++) {
        int x = xs[i], y = ys[i], a = canvas_area(mL, mR, pitch, x, y);
        if (a == 1) {
            out[i] = 0.0;
        } else if (a == 2) {
            out[i] = 1.0;
        } else if (a == 0) {
            out[i] = 0.5;
        } else {
            long long d1 = nearest_d2(mL, mR, pitch, H, W, x, y, 1, periodic);
            long long d2 = nearest_d2(mL, mR, pitch, H, W, x, y, 2, periodic);
            if (d1 < 0 && d2 < 0)
                out[i] = 0.5;
            else if (d1 < 0)
                out[i] = 1.0;
            else if (d2 < 0)
                out[i] = 0.0;
            else {
                double lmin = sqrt((double)d1), rmin = sqrt((double)d2);
                out[i] = lmin / (lmin + rmin);
            }
        }
    }
}

/* Bounding box of Area3 as {x, y, width, height}; {0, 0, 0, 0} if empty.
 * Rows: the first to the last row holding an Area3 pixel. Columns: on a
 * plain canvas the first to the last such column. On a periodic canvas the
 * columns form a circle and the box is the shortest run of consecutive
 * columns (wrapping past W - 1 to 0) that holds every Area3 column: it
 * starts right after the longest run of columns without an Area3 pixel
 * (of several longest, the one that starts at the smallest column; a run
 * that wraps starts at its column nearest W - 1) and w = W minus that run's
 * length, so x + w may exceed W; with no such run (every column holds an
 * Area3 pixel) the box starts at 0 with w = W. */
void orc_overlap_box(const uint8_t *mL, const uint8_t *mR, long pitch, int H, int W, int periodic, int32_t box[4])
{
    int x0 = W, y0 = H, x1 = -1, y1 = -1;
    char *occ = (char *)calloc((size_t)W, 1);
    for (int y = 0; y < H; y++)
        for (int x = 0; x < W; x++)
            if (canvas_area(mL, mR, pitch, x, y) == 3) {
                occ[x] = 1;
                if (x < x0) x0 = x;
                if (x > x1) x1 = x;
                if (y < y0) y0 = y;
                if (y > y1) y1 = y;
            }
    if (x1 < 0) {
        box[0] = box[1] = box[2] = box[3] = 0;
    } else {
        box[0] = x0;
        box[1] = y0;
        box[2] = x1 - x0 + 1;
        box[3] = y1 - y0 + 1;
        if (periodic) {
            /* every run of empty columns, by its first column s (the column
             * before it, circularly, holds an Area3 pixel) */
            int best_s = -1, best_len = 0;
            for (int s0 = 0; s0 < W; s0++) {
                if (occ[s0] || !occ[(s0 + W - 1) % W]) continue;
                int len = 0;
                while (len < W && !occ[(s0 + len) % W]) len++;
                if (len > best_len) {
                    best_len = len;
                    best_s = s0;
                }
            }
            if (best_len == 0) {
                box[0] = 0;
                box[2] = W;
            } else {
                box[0] = (best_s + best_len) % W;
                box[2] = W - best_len;
            }
        }
    }
    free(occ);
}

/* Code 1 over a canvas. L, R: double H x W x 3 canvas images. The flows
 * are box[3] x box[2] x 2 over the overlap box {x, y, w, h}: OverlappedL /
 * OverlappedR are the box's crops of L and R, and Area3 pixels are warped
 * and blended exactly as in orc_blend on that crop (samples clamped to the
 * crop, flow magnitude divided by the box extent across the seam), with
 * Blend taken from `blend` (H x W canvas array) or from eq. (1) if NULL.
 * Area1 copies L, Area2 copies R, every other pixel (and an Area3 pixel
 * outside the box, which has no flow) is 0. */
void orc_composite(const double *L, const double *R, const uint8_t *mL, const uint8_t *mR, long pitch, int H, int W,
                   int periodic, const double *flow_lr, const double *flow_rl, const int32_t box[4], int axis,
                   const double *blend, double kS, double kF, int mode, double *F, uint8_t *F8)
{
    int bx = box[0], by = box[1], bw = box[2], bh = box[3];
    long nb = (long)bw * bh;
    double *Lc = NULL, *Rc = NULL, *Bc = NULL, *Fc = NULL;
    if (nb > 0) {
        Lc = (double *)malloc(sizeof(double) * 3 * nb);
        Rc = (double *)malloc(sizeof(double) * 3 * nb);
        Bc = (double *)malloc(sizeof(double) * nb);
        Fc = (double *)malloc(sizeof(double) * 3 * nb);
        int32_t *xs = (int32_t *)malloc(sizeof(int32_t) * nb), *ys = (int32_t *)malloc(sizeof(int32_t) * nb);
        for (int y = 0; y < bh; y++)
            for (int x = 0; x < bw; x++) {
                /* crop column x is canvas column bx + x, modulo W on a periodic canvas */
                int cx = (x + bx) % W;
                long q = (long)y * bw + x, p = (long)(y + by) * W + cx;
                for (int c = 0; c < 3; c++) {
                    Lc[3 * q + c] = L[3 * p + c];
                    Rc[3 * q + c] = R[3 * p + c];
                }
                xs[q] = cx;
                ys[q] = y + by;
                if (blend) Bc[q] = blend[p];
            }
        if (!blend) orc_canvas_blend(mL, mR, pitch, H, W, periodic, nb, xs, ys, Bc);
        orc_blend(Lc, Rc, flow_lr, flow_rl, Bc, axis, bh, bw, kS, kF, mode, Fc, NULL);
        free(xs);
        free(ys);
    }
    for (int y = 0; y < H; y++)
        for (int x = 0; x < W; x++) {
            long p = (long)y * W + x;
            int a = canvas_area(mL, mR, pitch, x, y);
            int xb = x - bx;
            if (periodic && xb < 0) xb += W;
            int inbox = xb >= 0 && xb < bw && y >= by && y < by + bh;
            for (int c = 0; c < 3; c++) {
                double f = 0.0;
                if (a == 1)
                    f = L[3 * p + c];
                else if (a == 2)
                    f = R[3 * p + c];
                else if (a == 3 && inbox)
                    f = Fc[3 * ((long)(y - by) * bw + xb) + c];
                F[3 * p + c] = f;
                if (F8) {
                    double r = floor(f + 0.5);
                    F8[3 * p + c] = (uint8_t)(r < 0 ? 0 : (r > 255 ? 255 : r));
                }
            }
        }
    free(Lc);
    free(Rc);
    free(Bc);
    free(Fc);
}
