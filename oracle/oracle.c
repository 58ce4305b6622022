/*
 * Connectivity-counting oracle -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, obviously correct CPU implementation of the pass-through
 * connectivity matrix of FastCod (Bian, Shao, Zhuo, Gullapalli, Carass, Prince,
 * "FastCod: Fast Brain Connectivity in Diffusion Imaging", SPIE Medical Imaging
 * 2023).  Only the test suite, the package smoke check and the benchmark's CPU
 * baseline may call it.  The product path (the HIP library) never links, loads
 * or calls anything in this directory, and this file includes nothing from it.
 *
 * What is computed (Section 2 "Method", Alg. 2 with its passthrough and
 * loc2region functions and the C update; the abstract and Section 1 state the
 * reading used here: two regions are connected when one streamline passes
 * through both, wherever it starts or ends):
 *
 *   A streamline l is an ordered list of 3-D points p^1..p^T (Section 2).
 *   vox(p)  = ( floor(fl32(p_x + 0.5)), floor(fl32(p_y + 0.5)), floor(fl32(p_z + 0.5)) )
 *             with voxel centres at integer coordinates; a point whose voxel lies
 *             outside the X*Y*Z grid (or has a NaN/inf coordinate) touches nothing.
 *   I_l     = { roi[vox(p)] : p in l, vox(p) in grid, 0 <= roi[vox(p)] < N }
 *   M_l     = { lab[vox(p)] : p in l, vox(p) in grid, 0 <= lab[vox(p)] < M }
 *   C[i][m] = #{ l : i in I_l and m in M_l }          (C is N x M, row i = voxel v_i)
 *
 * Volumes are stored [Z][Y][X] with x fastest: lin = x + X*(y + Y*z).
 * With a coordinate scale s (the super-resolution transform of Section 3,
 * "Super-resolving connectivity features"), every coordinate is first replaced
 * by fl32(p * s); s = 1 leaves the points unchanged.
 *
 * Two variants follow the same conventions: oracle_count_endpoint (Alg. 2 as
 * printed, the target label read at the streamline's last point only) and
 * oracle_count_seed_endpoint (Alg. 1's count, one per streamline at its seed
 * row and end label).
 *
 * Readings taken where the paper is silent (rounding, out-of-grid points,
 * repeated visits, values outside [0,N) / [0,M)) are listed in the design notes
 * of the repository; each one is exercised by a test.
 *
 * Build: gcc -O2 -ffp-contract=off -fno-fast-math -shared -fPIC (no FMA
 * contraction, so p*s and +0.5 are two separately rounded float operations).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* Linear voxel index of one point, or -1 when the point touches no voxel of the grid. */
int64_t oracle_voxel(float px, float py, float pz, float scale, const int32_t dims[3])
{
    float p[3] = {px, py, pz};
    int64_t v[3];
    for (int k = 0; k < 3; ++k) {
        float q = p[k] * scale;        /* fl32(p * s); exact when s == 1 */
        float t = q + 0.5f;            /* fl32(q + 0.5), round to nearest even */
        float f = floorf(t);
        /* NaN fails both comparisons; the bound is compared in double so that
           grid sizes above 2^24 are still exact. */
        if (!(f >= 0.0f) || !((double)f < (double)dims[k]))
            return -1;
        v[k] = (int64_t)f;
    }
    return v[0] + (int64_t)dims[0] * (v[1] + (int64_t)dims[1] * v[2]);
}

static int cmp_i32(const void *a, const void *b)
{
    int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
    return (x > y) - (x < y);
}

/* Sort and drop repeats; returns the number of distinct values. */
static int64_t sort_unique(int32_t *v, int64_t n)
{
    if (n == 0)
        return 0;
    qsort(v, (size_t)n, sizeof(int32_t), cmp_i32);
    int64_t k = 1;
    for (int64_t j = 1; j < n; ++j)
        if (v[j] != v[k - 1])
            v[k++] = v[j];
    return k;
}

/*
 * Pass-through connectivity matrix.
 *   points  [P][3] float32, streamline s = points[offsets[s] .. offsets[s+1])
 *   offsets [S+1] int64, offsets[0] = 0, nondecreasing
 *   roi, lab [Z][Y][X] int32 volumes, dims = {X, Y, Z}
 *   C       [N][M] int64, overwritten
 * Returns 0, or -1 on bad arguments / out of memory.
 */
int oracle_count(const float *points, const int64_t *offsets, int64_t S,
                 const int32_t *roi, const int32_t *lab, const int32_t dims[3],
                 int32_t N, int32_t M, float scale, int64_t *C)
{
    if (S < 0 || N < 1 || M < 1 || !C || !dims)
        return -1;
    memset(C, 0, sizeof(int64_t) * (size_t)N * (size_t)M);

    int64_t cap = 0;
    int32_t *I = NULL, *L = NULL;
    for (int64_t s = 0; s < S; ++s) {
        int64_t a = offsets[s], b = offsets[s + 1];
        int64_t T = b - a;
        if (T <= 0)
            continue;                       /* an empty streamline touches nothing */
        if (T > cap) {
            free(I);
            free(L);
            cap = T;
            I = (int32_t *)malloc(sizeof(int32_t) * (size_t)cap);
            L = (int32_t *)malloc(sizeof(int32_t) * (size_t)cap);
            if (!I || !L) {
                free(I);
                free(L);
                return -1;
            }
        }
        /* passthrough(l, V) and loc2region(p, R) for every point of l */
        int64_t nI = 0, nL = 0;
        for (int64_t j = a; j < b; ++j) {
            const float *p = points + 3 * j;
            int64_t lin = oracle_voxel(p[0], p[1], p[2], scale, dims);
            if (lin < 0)
                continue;
            int32_t r = roi[lin];
            int32_t m = lab[lin];
            if (r >= 0 && r < N)
                I[nI++] = r;
            if (m >= 0 && m < M)
                L[nL++] = m;
        }
        /* the sets I_l and M_l: each distinct value once */
        nI = sort_unique(I, nI);
        nL = sort_unique(L, nL);
        /* C(i, m) += 1 for every i in I_l and m in M_l */
        for (int64_t x = 0; x < nI; ++x)
            for (int64_t y = 0; y < nL; ++y)
                C[(int64_t)I[x] * M + L[y]] += 1;
    }
    free(I);
    free(L);
    return 0;
}

/* Row of the voxel holding one point, or -1 (no voxel, or an ROI value outside [0, N)). */
static int32_t row_at(const float *p, float scale, const int32_t *roi, const int32_t dims[3], int32_t N)
{
    int64_t lin = oracle_voxel(p[0], p[1], p[2], scale, dims);
    if (lin < 0)
        return -1;
    return (roi[lin] >= 0 && roi[lin] < N) ? roi[lin] : -1;
}

/* Label of the voxel holding one point (loc2region), or -1 (no voxel, or a value outside [0, M)). */
static int32_t label_at(const float *p, float scale, const int32_t *lab, const int32_t dims[3], int32_t M)
{
    int64_t lin = oracle_voxel(p[0], p[1], p[2], scale, dims);
    if (lin < 0)
        return -1;
    return (lab[lin] >= 0 && lab[lin] < M) ? lab[lin] : -1;
}

/*
 * Endpoint-label matrix: Alg. 2 as printed, where loc2region reads only the
 * last point p^T of the streamline while passthrough reads all of them.
 *   I_l     = the ROI rows passed through, as in oracle_count;
 *   E_l     = { label of p^T }, empty when p^T has no voxel or no label;
 *             with both_ends, E_l also holds the label of the first point p^1
 *             (a set: a label at both ends is counted once);
 *   C[i][m] = #{ l : i in I_l and m in E_l }.
 * Arguments as oracle_count.
 */
int oracle_count_endpoint(const float *points, const int64_t *offsets, int64_t S,
                          const int32_t *roi, const int32_t *lab, const int32_t dims[3],
                          int32_t N, int32_t M, float scale, int both_ends, int64_t *C)
{
    if (S < 0 || N < 1 || M < 1 || !C || !dims)
        return -1;
    memset(C, 0, sizeof(int64_t) * (size_t)N * (size_t)M);
    int64_t cap = 0;
    int32_t *I = NULL;
    for (int64_t s = 0; s < S; ++s) {
        int64_t a = offsets[s], b = offsets[s + 1];
        if (b <= a)
            continue;
        int32_t e_last = label_at(points + 3 * (b - 1), scale, lab, dims, M);
        int32_t e_first = both_ends ? label_at(points + 3 * a, scale, lab, dims, M) : -1;
        if (e_first == e_last)
            e_first = -1;                   /* the set E_l holds a shared label once */
        if (e_last < 0 && e_first < 0)
            continue;
        if (b - a > cap) {
            free(I);
            cap = b - a;
            I = (int32_t *)malloc(sizeof(int32_t) * (size_t)cap);
            if (!I)
                return -1;
        }
        int64_t nI = 0;
        for (int64_t j = a; j < b; ++j) {
            int32_t r = row_at(points + 3 * j, scale, roi, dims, N);
            if (r >= 0)
                I[nI++] = r;
        }
        nI = sort_unique(I, nI);
        for (int64_t x = 0; x < nI; ++x) {
            if (e_last >= 0)
                C[(int64_t)I[x] * M + e_last] += 1;
            if (e_first >= 0)
                C[(int64_t)I[x] * M + e_first] += 1;
        }
    }
    free(I);
    return 0;
}

/*
 * Seed-to-endpoint counting, the analogue of Alg. 1 on the same streamlines:
 * the streamline grown from a seed in voxel v_i adds one to C(v_i,
 * loc2region(p^T)).  The seed is the streamline's first point p^1:
 *   C[i][m] = #{ l : row of p^1 is i and label of p^T is m }.
 * Arguments as oracle_count.
 */
int oracle_count_seed_endpoint(const float *points, const int64_t *offsets, int64_t S,
                               const int32_t *roi, const int32_t *lab, const int32_t dims[3],
                               int32_t N, int32_t M, float scale, int64_t *C)
{
    if (S < 0 || N < 1 || M < 1 || !C || !dims)
        return -1;
    memset(C, 0, sizeof(int64_t) * (size_t)N * (size_t)M);
    for (int64_t s = 0; s < S; ++s) {
        int64_t a = offsets[s], b = offsets[s + 1];
        if (b <= a)
            continue;
        int32_t seed_row = row_at(points + 3 * a, scale, roi, dims, N);
        int32_t end_label = label_at(points + 3 * (b - 1), scale, lab, dims, M);
        if (seed_row >= 0 && end_label >= 0)
            C[(int64_t)seed_row * M + end_label] += 1;
    }
    return 0;
}

/*
 * Parcellation outputs of a connectivity matrix (Section 3, "Pie-glyphs"): the
 * "single colour" map shows, for each source voxel (row i), the target region
 * it is most strongly connected to, and a pie-glyph shows its relative
 * connection strength to every region.
 *   sums[i]    = sum over m of C[i][m]  (int64)
 *   label[i]   = the smallest m with C[i][m] equal to the row's maximum, or -1
 *                when no entry of the row is positive
 *   frac[i][m] = C[i][m] / sums[i], the quotient of the two integers taken in
 *                double and rounded to float; 0 when sums[i] <= 0
 * C is [N][M] int64; label [N], frac [N][M] and sums [N] are written.
 */
int oracle_parcellate(const int64_t *C, int32_t N, int32_t M, int32_t *label, float *frac, int64_t *sums)
{
    if (N < 0 || M < 1 || !C || !label || !frac || !sums)
        return -1;
    for (int64_t i = 0; i < N; ++i) {
        const int64_t *row = C + i * M;
        int64_t total = 0;
        int32_t best = -1;
        for (int32_t m = 0; m < M; ++m) {
            total += row[m];
            if (row[m] > 0 && (best < 0 || row[m] > row[best]))
                best = m;
        }
        sums[i] = total;
        label[i] = best;
        for (int32_t m = 0; m < M; ++m)
            frac[i * M + m] = total > 0 ? (float)((double)row[m] / (double)total) : 0.0f;
    }
    return 0;
}

/*
 * Pass-through matrix of upsampled streamlines (Section 3, "Super-resolving
 * connectivity features": evenly spaced points are inserted between every two
 * neighbouring points of a streamline, so that the spacing falls below half a
 * voxel of the grid where connectivity is computed).  With the scaled points
 * q_k = fl32(p_k * s) and a factor u >= 1, a streamline is counted as
 *   q_1, y_{1,1} .. y_{1,u-1}, q_2, y_{2,1} .. y_{2,u-1}, q_3, ..., q_T
 *   y_{k,t} = fl32(q_k + fl32(a_t * fl32(q_{k+1} - q_k))),   a_t = fl32(t / u),
 * every operation rounded to float on its own (no fused multiply-add), per
 * coordinate.  Then I_l, M_l and C exactly as in oracle_count; u = 1 is
 * oracle_count itself.
 */
int oracle_count_upsampled(const float *points, const int64_t *offsets, int64_t S,
                           const int32_t *roi, const int32_t *lab, const int32_t dims[3],
                           int32_t N, int32_t M, float scale, int32_t u, int64_t *C)
{
    if (S < 0 || N < 1 || M < 1 || u < 1 || !C || !dims)
        return -1;
    memset(C, 0, sizeof(int64_t) * (size_t)N * (size_t)M);
    int64_t cap = 0;
    float *D = NULL;                        /* the upsampled streamline, scaled, [len][3] */
    int32_t *I = NULL, *L = NULL;
    for (int64_t s = 0; s < S; ++s) {
        int64_t a = offsets[s], b = offsets[s + 1];
        int64_t T = b - a;
        if (T <= 0)
            continue;
        int64_t len = T + (T - 1) * (int64_t)(u - 1);
        if (len > cap) {
            free(D);
            free(I);
            free(L);
            cap = len;
            D = (float *)malloc(sizeof(float) * 3 * (size_t)cap);
            I = (int32_t *)malloc(sizeof(int32_t) * (size_t)cap);
            L = (int32_t *)malloc(sizeof(int32_t) * (size_t)cap);
            if (!D || !I || !L) {
                free(D);
                free(I);
                free(L);
                return -1;
            }
        }
        int64_t n = 0;
        for (int64_t j = a; j < b; ++j) {
            for (int k = 0; k < 3; ++k)
                D[3 * n + k] = points[3 * j + k] * scale;              /* q_j */
            ++n;
            if (j + 1 == b)
                break;                                              /* nothing after the last point */
            for (int32_t t = 1; t < u; ++t) {
                float at = (float)t / (float)u;                     /* a_t = fl32(t / u) */
                for (int k = 0; k < 3; ++k) {
                    float qk = points[3 * j + k] * scale;
                    float qn = points[3 * (j + 1) + k] * scale;
                    float d = qn - qk;
                    float e = at * d;
                    D[3 * n + k] = qk + e;
                }
                ++n;
            }
        }
        /* the upsampled points are already scaled: look them up with scale 1 (exact) */
        int64_t nI = 0, nL = 0;
        for (int64_t j = 0; j < n; ++j) {
            int64_t lin = oracle_voxel(D[3 * j], D[3 * j + 1], D[3 * j + 2], 1.0f, dims);
            if (lin < 0)
                continue;
            if (roi[lin] >= 0 && roi[lin] < N)
                I[nI++] = roi[lin];
            if (lab[lin] >= 0 && lab[lin] < M)
                L[nL++] = lab[lin];
        }
        nI = sort_unique(I, nI);
        nL = sort_unique(L, nL);
        for (int64_t x = 0; x < nI; ++x)
            for (int64_t y = 0; y < nL; ++y)
                C[(int64_t)I[x] * M + L[y]] += 1;
    }
    free(D);
    free(I);
    free(L);
    return 0;
}
