/*
 * Plain FP64 CPU oracle for the narrow-band sparse-grid hot path.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may call, link or
 * load this file; only the tests, the smoke check and the benchmark's CPU
 * baseline leg use it.  It shares no code, header or table with the HIP
 * library: every quantity is written out here from its definition, on a
 * dense N^3 grid (N = 4M data points per axis, x fastest), in double
 * precision, with plain loops.
 *
 * Definitions followed (section numbers are those of the paper, "Contiguous
 * Storage of Grid Data for Heterogeneous Computing"):
 *   - activation: a coarse cell is core when the distance at its centre is
 *     below the coarse cell size; inner when it is not core but one of its
 *     nearest neighbours is core (Sec. 7.1, steps 1-2);
 *   - numbering: activated cells sorted by spatial position (linear index),
 *     after two reserved far-field packages, 0 = negative (inside) and
 *     1 = positive (outside) (Sec. 5 and Sec. 7.1, step 3);
 *   - neighbourhood: a 3x3x3 table of neighbour package indices per package,
 *     far-field packages neighbouring themselves (Sec. 5.2, Sec. 7.1 step 5);
 *   - index shift: Sec. 5.2, Listing 2;
 *   - central difference: Sec. 7.3, Listing 5 (plain average of the two
 *     one-sided differences);
 *   - trilinear grid-to-particle interpolation: Sec. 8.
 * Steps the paper names but does not define (upwind reinitialisation, the
 * near-surface kernel integral, the MLP surrogate) follow the readings the
 * design document lists; each function says which.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define FAR_NEG 0u
#define FAR_POS 1u
#define NO_CELL 0xFFFFFFFFu

static inline int64_t lin3(int64_t i, int64_t j, int64_t k, int64_t n) { return i + n * (j + n * k); }

/* ------------------------------------------------------------------------ */
/* Activation (Sec. 7.1 steps 1-2).  type[c]: 0 inactive, 1 core, 2 inner.   */
/* `d` is the distance at each coarse-cell centre (float, taken exactly).    */
/* ------------------------------------------------------------------------ */
void orc_classify(int32_t M, double lc, const float *d, uint8_t *type)
{
    const int64_t n = (int64_t)M * M * M;
    uint8_t *core = (uint8_t *)calloc((size_t)n, 1);
    for (int64_t c = 0; c < n; ++c) core[c] = fabs((double)d[c]) < lc;
    for (int64_t z = 0; z < M; ++z)
        for (int64_t y = 0; y < M; ++y)
            for (int64_t x = 0; x < M; ++x) {
                int64_t c = lin3(x, y, z, M);
                if (core[c]) { type[c] = 1; continue; }
                int found = 0;
                for (int dz = -1; dz <= 1 && !found; ++dz)
                    for (int dy = -1; dy <= 1 && !found; ++dy)
                        for (int dx = -1; dx <= 1 && !found; ++dx) {
                            if (!dx && !dy && !dz) continue;
                            int64_t xx = x + dx, yy = y + dy, zz = z + dz;
                            if (xx < 0 || yy < 0 || zz < 0 || xx >= M || yy >= M || zz >= M) continue;
                            if (core[lin3(xx, yy, zz, M)]) found = 1;
                        }
                type[c] = found ? 2 : 0;
            }
    free(core);
}

/* ------------------------------------------------------------------------ */
/* Consistency (sign) correction of a layer's distances (Sec. 7.2), the coarse */
/* step on the mesh cells: only the signs of cells near the surface (core,    */
/* |d| < lc) are used as given; every other cell gets its sign by diffusion   */
/* from them.  Rounds of simultaneous updates: a cell without a sign yet      */
/* takes one when a face neighbour has one, positive if any such neighbour is */
/* positive, else negative; rounds repeat until one changes nothing.  Output: */
/* core cells keep d; cells that received a sign get |d| with it; cells no    */
/* diffusion reaches keep d.  Returns the number of rounds that changed a    */
/* cell.                                                                      */
/* ------------------------------------------------------------------------ */
int32_t orc_correct_signs(int32_t M, double lc, const float *d, float *out)
{
    const int64_t n = (int64_t)M * M * M;
    uint8_t *state = (uint8_t *)malloc((size_t)n);    /* 0 no sign, 1 negative, 2 positive */
    uint8_t *next = (uint8_t *)malloc((size_t)n);
    for (int64_t c = 0; c < n; ++c)
        state[c] = fabs((double)d[c]) < lc ? (d[c] < 0.0f ? 1 : 2) : 0;
    int32_t rounds = 0;
    for (;;) {
        int changed = 0;
#pragma omp parallel for schedule(static) reduction(| : changed)
        for (int64_t z = 0; z < M; ++z)
            for (int64_t y = 0; y < M; ++y)
                for (int64_t x = 0; x < M; ++x) {
                    const int64_t c = lin3(x, y, z, M);
                    next[c] = state[c];
                    if (state[c]) continue;
                    int pos = 0, neg = 0;
                    const int64_t nx[6] = {x - 1, x + 1, x, x, x, x}, ny[6] = {y, y, y - 1, y + 1, y, y},
                                  nz[6] = {z, z, z, z, z - 1, z + 1};
                    for (int f = 0; f < 6; ++f) {
                        if (nx[f] < 0 || ny[f] < 0 || nz[f] < 0 || nx[f] >= M || ny[f] >= M || nz[f] >= M) continue;
                        const uint8_t v = state[lin3(nx[f], ny[f], nz[f], M)];
                        pos |= v == 2;
                        neg |= v == 1;
                    }
                    if (pos || neg) {
                        next[c] = pos ? 2 : 1;
                        changed = 1;
                    }
                }
        uint8_t *t = state;
        state = next;
        next = t;
        if (!changed) break;
        ++rounds;
    }
    for (int64_t c = 0; c < n; ++c) {
        const int core = fabs((double)d[c]) < lc;
        if (core || state[c] == 0) out[c] = d[c];
        else out[c] = state[c] == 2 ? fabsf(d[c]) : -fabsf(d[c]);
    }
    free(state);
    free(next);
    return rounds;
}

/* ------------------------------------------------------------------------ */
/* Numbering (Sec. 5 and Sec. 7.1 step 3).  Returns P, the number of         */
/* activated packages.  pkg_cell / pkg_type must hold M^3 + 2 entries.       */
/* ------------------------------------------------------------------------ */
int64_t orc_number(int32_t M, const float *d, const uint8_t *type,
                   uint32_t *cell_pkg, uint32_t *pkg_cell, uint8_t *pkg_type)
{
    const int64_t n = (int64_t)M * M * M;
    int64_t k = 0;
    pkg_cell[FAR_NEG] = pkg_cell[FAR_POS] = NO_CELL;
    pkg_type[FAR_NEG] = pkg_type[FAR_POS] = 0;
    for (int64_t c = 0; c < n; ++c) {
        if (type[c]) {
            cell_pkg[c] = (uint32_t)(2 + k);
            pkg_cell[2 + k] = (uint32_t)c;
            pkg_type[2 + k] = type[c];
            ++k;
        } else {
            cell_pkg[c] = (d[c] < 0.0f) ? FAR_NEG : FAR_POS;
        }
    }
    return k;
}

/* ------------------------------------------------------------------------ */
/* Neighbour table (Sec. 5.2; far field neighbours itself, Sec. 7.1 step 5). */
/* Slot s = (dx+1) + 3(dy+1) + 9(dz+1).  Out-of-domain neighbours read the   */
/* positive far field.                                                       */
/* ------------------------------------------------------------------------ */
void orc_neighbours(int32_t M, const uint32_t *cell_pkg, const uint32_t *pkg_cell,
                    int64_t n_pkg_total, uint32_t *nbr)
{
    for (int s = 0; s < 27; ++s) { nbr[FAR_NEG * 27 + s] = FAR_NEG; nbr[FAR_POS * 27 + s] = FAR_POS; }
    for (int64_t p = 2; p < n_pkg_total; ++p) {
        int64_t c = pkg_cell[p];
        int64_t x = c % M, y = (c / M) % M, z = c / ((int64_t)M * M);
        for (int dz = -1; dz <= 1; ++dz)
            for (int dy = -1; dy <= 1; ++dy)
                for (int dx = -1; dx <= 1; ++dx) {
                    int s = (dx + 1) + 3 * (dy + 1) + 9 * (dz + 1);
                    int64_t xx = x + dx, yy = y + dy, zz = z + dz;
                    uint32_t v = FAR_POS;
                    if (xx >= 0 && yy >= 0 && zz >= 0 && xx < M && yy < M && zz < M)
                        v = cell_pkg[lin3(xx, yy, zz, M)];
                    nbr[p * 27 + s] = v;
                }
    }
}

/* Index shift of Sec. 5.2 (Listing 2) for one axis and package size 4:       */
/* neighbour slot = (s + 4) / 4, data index = s + 4 - 4 * slot.                */
void orc_index_shift(int32_t s, int32_t *slot, int32_t *data)
{
    *slot = (s + 4) / 4;
    *data = s + 4 - 4 * (*slot);
}

/* ------------------------------------------------------------------------ */
/* Dense-field helpers.  Reads outside [0, N)^3 return the positive far-field */
/* value B.                                                                  */
/* ------------------------------------------------------------------------ */
static inline double rd(const double *f, int64_t N, int64_t i, int64_t j, int64_t k, double B)
{
    if (i < 0 || j < 0 || k < 0 || i >= N || j >= N || k >= N) return B;
    return f[lin3(i, j, k, N)];
}

/* ------------------------------------------------------------------------ */
/* Reinitialisation: n_iter Jacobi sweeps of the Sussman-Smereka-Osher       */
/* equation phi_t + S(phi)(|grad phi| - 1) = 0 with Godunov upwinding, over   */
/* the listed active data points only (all other points keep their value).   */
/*   S = phi / sqrt(phi^2 + h^2), dt = h / 2,                                 */
/*   D- = (phi_p - phi_{p-e}) / h, D+ = (phi_{p+e} - phi_p) / h,              */
/*   S > 0: a^2 = max(max(D-,0)^2, min(D+,0)^2)                               */
/*   S < 0: a^2 = max(min(D-,0)^2, max(D+,0)^2)                               */
/*   phi' = phi - dt S (sqrt(sum a^2) - 1)                                    */
/* phi and work are dense N^3 arrays; the result ends in phi.                */
/* ------------------------------------------------------------------------ */
void orc_reinit(int32_t N, double h, double B, const int64_t *active, int64_t n_active,
                double *phi, double *work, int32_t n_iter)
{
    const int64_t n = (int64_t)N * N * N;
    const double dt = 0.5 * h;
    memcpy(work, phi, (size_t)n * sizeof(double));
    double *src = phi, *dst = work;
    for (int32_t it = 0; it < n_iter; ++it) {
#pragma omp parallel for schedule(static)
        for (int64_t q = 0; q < n_active; ++q) {
            int64_t l = active[q];
            int64_t i = l % N, j = (l / N) % N, k = l / ((int64_t)N * N);
            double p0 = src[l];
            double S = p0 / sqrt(p0 * p0 + h * h);
            double nb[3][2] = {
                {rd(src, N, i - 1, j, k, B), rd(src, N, i + 1, j, k, B)},
                {rd(src, N, i, j - 1, k, B), rd(src, N, i, j + 1, k, B)},
                {rd(src, N, i, j, k - 1, B), rd(src, N, i, j, k + 1, B)}};
            double sum = 0.0;
            for (int a = 0; a < 3; ++a) {
                double dm = (p0 - nb[a][0]) / h, dp = (nb[a][1] - p0) / h;
                double x, y;
                if (S > 0) { x = fmax(dm, 0.0); y = fmin(dp, 0.0); }
                else       { x = fmin(dm, 0.0); y = fmax(dp, 0.0); }
                sum += fmax(x * x, y * y);
            }
            dst[l] = (S == 0.0) ? p0 : p0 - dt * S * (sqrt(sum) - 1.0);
        }
        double *t = src; src = dst; dst = t;
    }
    if (src != phi) memcpy(phi, src, (size_t)n * sizeof(double));
}

/* ------------------------------------------------------------------------ */
/* Central-difference gradient (Listing 5 with the plain average):            */
/* g = (phi_{p+e} - phi_{p-e}) / (2h) at the listed active points; the caller */
/* zero-fills every other point.  g is three dense arrays gx, gy, gz.         */
/* ------------------------------------------------------------------------ */
void orc_gradient(int32_t N, double h, double B, const int64_t *active, int64_t n_active,
                  const double *phi, double *gx, double *gy, double *gz)
{
#pragma omp parallel for schedule(static)
    for (int64_t q = 0; q < n_active; ++q) {
        int64_t l = active[q];
        int64_t i = l % N, j = (l / N) % N, k = l / ((int64_t)N * N);
        gx[l] = (rd(phi, N, i + 1, j, k, B) - rd(phi, N, i - 1, j, k, B)) / (2.0 * h);
        gy[l] = (rd(phi, N, i, j + 1, k, B) - rd(phi, N, i, j - 1, k, B)) / (2.0 * h);
        gz[l] = (rd(phi, N, i, j, k + 1, B) - rd(phi, N, i, j, k - 1, B)) / (2.0 * h);
    }
}

/* ------------------------------------------------------------------------ */
/* Consistency (sign) correction, the refined step on the data packages      */
/* (Sec. 7.2): on a refined layer the operation is limited to the inner       */
/* packages.  The points of core packages keep their sign, like the core     */
/* cells of the coarse step, and so do points outside the band (the far-field */
/* constant of their cell; reads outside the domain are the positive far     */
/* field).  The points of inner packages (`inner`, a list of linear indices)  */
/* get their sign by diffusion over face neighbours, in rounds of            */
/* simultaneous updates (positive if any decided neighbour is positive, else */
/* negative), until a round changes nothing; they take |phi| with that sign, */
/* or keep phi if no diffusion reaches them.  Returns the number of rounds   */
/* that decided a point.                                                      */
/* ------------------------------------------------------------------------ */
int32_t orc_correct_point_signs(int32_t N, const int64_t *inner, int64_t n_inner, const double *phi, double *out)
{
    const int64_t n = (int64_t)N * N * N;
    uint8_t *state = (uint8_t *)malloc((size_t)n), *next = (uint8_t *)malloc((size_t)n);
    for (int64_t c = 0; c < n; ++c) state[c] = phi[c] < 0.0 ? 1 : 2;
    for (int64_t q = 0; q < n_inner; ++q) state[inner[q]] = 0;
    int32_t rounds = 0;
    for (;;) {
        int changed = 0;
        memcpy(next, state, (size_t)n);
#pragma omp parallel for schedule(static) reduction(| : changed)
        for (int64_t q = 0; q < n_inner; ++q) {
            const int64_t c = inner[q];
            if (state[c]) continue;
            const int64_t i = c % N, j = (c / N) % N, k = c / ((int64_t)N * N);
            const int64_t nx[6] = {i - 1, i + 1, i, i, i, i}, ny[6] = {j, j, j - 1, j + 1, j, j},
                          nz[6] = {k, k, k, k, k - 1, k + 1};
            int pos = 0, neg = 0;
            for (int f = 0; f < 6; ++f) {
                uint8_t v;
                if (nx[f] < 0 || ny[f] < 0 || nz[f] < 0 || nx[f] >= N || ny[f] >= N || nz[f] >= N) v = 2;
                else v = state[lin3(nx[f], ny[f], nz[f], N)];
                pos |= v == 2;
                neg |= v == 1;
            }
            if (pos || neg) {
                next[c] = pos ? 2 : 1;
                changed = 1;
            }
        }
        uint8_t *t = state;
        state = next;
        next = t;
        if (!changed) break;
        ++rounds;
    }
    memcpy(out, phi, (size_t)n * sizeof(double));
    for (int64_t q = 0; q < n_inner; ++q) {
        const int64_t c = inner[q];
        if (state[c]) out[c] = state[c] == 2 ? fabs(phi[c]) : -fabs(phi[c]);
    }
    free(state);
    free(next);
    return rounds;
}

/* ------------------------------------------------------------------------ */
/* The stencil operation of the paper's timing test (Sec. 9, Tab. 1): the     */
/* seven-point Laplacian (sum of the six face neighbours - 6 phi) / h^2 at    */
/* the listed active points; out-of-band neighbours read their far-field      */
/* constant.  The caller zero-fills every other point.                        */
/* ------------------------------------------------------------------------ */
void orc_laplacian(int32_t N, double h, double B, const int64_t *active, int64_t n_active,
                   const double *phi, double *out)
{
#pragma omp parallel for schedule(static)
    for (int64_t q = 0; q < n_active; ++q) {
        int64_t l = active[q];
        int64_t i = l % N, j = (l / N) % N, k = l / ((int64_t)N * N);
        double s = rd(phi, N, i - 1, j, k, B) + rd(phi, N, i + 1, j, k, B)
                 + rd(phi, N, i, j - 1, k, B) + rd(phi, N, i, j + 1, k, B)
                 + rd(phi, N, i, j, k - 1, B) + rd(phi, N, i, j, k + 1, B);
        out[l] = (s - 6.0 * phi[l]) / (h * h);
    }
}

/* ------------------------------------------------------------------------ */
/* Grid-to-particle probe (Sec. 8): trilinear interpolation of phi and g over */
/* the 8 data points around the particle, then n = g / |g| (0 when g = 0).    */
/* Per axis: u = x / h, s = u - 1/2, i0 = clamp(floor(s), 0, N-2),            */
/* t = clamp(s - i0, 0, 1).  The particle's package is the coarse cell        */
/* clamp(floor(u / 4), 0, M-1) that contains it; when that cell is not        */
/* activated its package is a far-field one, whose neighbours are itself, so  */
/* every corner reads the far-field constant and g = 0.  g_out (nullable)     */
/* receives the interpolated g.                                               */
/* ------------------------------------------------------------------------ */
void orc_probe(int32_t N, double h, double B, const uint32_t *cell_pkg,
               const double *phi, const double *gx, const double *gy, const double *gz,
               const double *pos, int64_t n, double *phi_out, double *nrm_out, double *g_out)
{
    const int64_t M = N / 4;
#pragma omp parallel for schedule(static)
    for (int64_t q = 0; q < n; ++q) {
        int64_t i0[3], cc[3];
        double t[3];
        for (int a = 0; a < 3; ++a) {
            double u = pos[3 * q + a] / h;
            double s = u - 0.5;
            double f = floor(s);
            if (f < 0) f = 0;
            if (f > N - 2) f = N - 2;
            i0[a] = (int64_t)f;
            double tt = s - f;
            t[a] = tt < 0 ? 0 : (tt > 1 ? 1 : tt);
            double cf = floor(u / 4.0);
            if (cf < 0) cf = 0;
            if (cf > M - 1) cf = M - 1;
            cc[a] = (int64_t)cf;
        }
        uint32_t home = cell_pkg[lin3(cc[0], cc[1], cc[2], M)];
        if (home < 2) {
            phi_out[q] = (home == FAR_NEG) ? -B : B;
            nrm_out[3 * q] = nrm_out[3 * q + 1] = nrm_out[3 * q + 2] = 0.0;
            if (g_out) g_out[3 * q] = g_out[3 * q + 1] = g_out[3 * q + 2] = 0.0;
            continue;
        }
        double v = 0, g[3] = {0, 0, 0};
        for (int b = 0; b < 8; ++b) {
            int bx = b & 1, by = (b >> 1) & 1, bz = (b >> 2) & 1;
            double w = (bx ? t[0] : 1 - t[0]) * (by ? t[1] : 1 - t[1]) * (bz ? t[2] : 1 - t[2]);
            int64_t l = lin3(i0[0] + bx, i0[1] + by, i0[2] + bz, N);
            v += w * phi[l];
            g[0] += w * gx[l];
            g[1] += w * gy[l];
            g[2] += w * gz[l];
        }
        double gn = sqrt(g[0] * g[0] + g[1] * g[1] + g[2] * g[2]);
        phi_out[q] = v;
        for (int a = 0; a < 3; ++a) nrm_out[3 * q + a] = gn > 0 ? g[a] / gn : 0.0;
        if (g_out) for (int a = 0; a < 3; ++a) g_out[3 * q + a] = g[a];
    }
}

/* ------------------------------------------------------------------------ */
/* Grid-to-particle coupling of the integral field (Sec. 8): the field        */
/* (K_W, h K_grad) is interpolated trilinearly to the particle position.      */
/* Same corner and weight rules as orc_probe; f holds the four components as  */
/* [4][N^3].  When the particle's home coarse cell is not activated, every    */
/* corner reads the constants of that far-field package, far[4 * side]        */
/* (side 0 negative, 1 positive).  out is [n][4].                             */
/* ------------------------------------------------------------------------ */
void orc_probe_field(int32_t N, double h, const uint32_t *cell_pkg, const double *f, const double *far,
                     const double *pos, int64_t n, double *out)
{
    const int64_t M = N / 4, NN = (int64_t)N * N * N;
#pragma omp parallel for schedule(static)
    for (int64_t q = 0; q < n; ++q) {
        int64_t i0[3], cc[3];
        double t[3];
        for (int a = 0; a < 3; ++a) {
            double u = pos[3 * q + a] / h;
            double s = u - 0.5;
            double fl = floor(s);
            if (fl < 0) fl = 0;
            if (fl > N - 2) fl = N - 2;
            i0[a] = (int64_t)fl;
            double tt = s - fl;
            t[a] = tt < 0 ? 0 : (tt > 1 ? 1 : tt);
            double cf = floor(u / 4.0);
            if (cf < 0) cf = 0;
            if (cf > M - 1) cf = M - 1;
            cc[a] = (int64_t)cf;
        }
        uint32_t home = cell_pkg[lin3(cc[0], cc[1], cc[2], M)];
        for (int c = 0; c < 4; ++c) {
            if (home < 2) { out[4 * q + c] = far[4 * home + c]; continue; }
            double v = 0;
            for (int b = 0; b < 8; ++b) {
                int bx = b & 1, by = (b >> 1) & 1, bz = (b >> 2) & 1;
                double w = (bx ? t[0] : 1 - t[0]) * (by ? t[1] : 1 - t[1]) * (bz ? t[2] : 1 - t[2]);
                v += w * f[c * NN + lin3(i0[0] + bx, i0[1] + by, i0[2] + bz, N)];
            }
            out[4 * q + c] = v;
        }
    }
}

/* ------------------------------------------------------------------------ */
/* Plane-cube volume fraction: the fraction of the cube u in [-1/2, 1/2]^3     */
/* where a + g.u > 0, written as the iterated integral of the indicator and   */
/* evaluated exactly: the innermost length is piecewise linear in the middle  */
/* variable and the area is piecewise quadratic in the outer one, with known  */
/* breakpoints, so the midpoint rule and 2-point Gauss-Legendre are exact on  */
/* each piece.  With g = 0 the fraction is 1, 0 or 1/2 for a >, <, = 0.       */
/* ------------------------------------------------------------------------ */
static double len1(double c, double g)       /* |{w in [0,1] : g w > c}| */
{
    if (g > 0) { double v = 1.0 - c / g; return v < 0 ? 0 : (v > 1 ? 1 : v); }
    if (g < 0) { double v = c / g;       return v < 0 ? 0 : (v > 1 ? 1 : v); }
    return c < 0 ? 1.0 : (c > 0 ? 0.0 : 0.5);
}

static int cmp_double(const void *a, const void *b)
{
    double x = *(const double *)a, y = *(const double *)b;
    return (x > y) - (x < y);
}

static int pieces(double *bp, int n)               /* sort breakpoints in [0,1] */
{
    qsort(bp, (size_t)n, sizeof(double), cmp_double);
    return n;
}

static double area2(double c, double g1, double g2)   /* |{w in [0,1]^2 : g1 w1 + g2 w2 > c}| */
{
    double bp[4] = {0.0, 1.0};
    int n = 2;
    if (g2 != 0.0) {
        double z[2] = {0.0, g1};
        for (int q = 0; q < 2; ++q) {
            double w = (c - z[q]) / g2;
            if (w > 0.0 && w < 1.0) bp[n++] = w;
        }
    }
    n = pieces(bp, n);
    double s = 0.0;
    for (int q = 0; q + 1 < n; ++q) {
        double a = bp[q], b = bp[q + 1];
        if (b <= a) continue;
        s += (b - a) * len1(c - g2 * 0.5 * (a + b), g1);
    }
    return s;
}

double orc_plane_cube_fraction(double a, double g1, double g2, double g3)
{
    /* w = u + 1/2 in [0,1]^3:  g.w > c  with  c = (g1 + g2 + g3)/2 - a */
    double c = 0.5 * (g1 + g2 + g3) - a;
    if (g1 == 0.0 && g2 == 0.0 && g3 == 0.0) return a > 0 ? 1.0 : (a < 0 ? 0.0 : 0.5);
    double bp[6] = {0.0, 1.0};
    int n = 2;
    if (g3 != 0.0) {
        double z[4] = {0.0, g1, g2, g1 + g2};
        for (int q = 0; q < 4; ++q) {
            double w = (c - z[q]) / g3;
            if (w > 0.0 && w < 1.0) bp[n++] = w;
        }
    }
    n = pieces(bp, n);
    const double r = 0.5 / sqrt(3.0);
    double s = 0.0;
    for (int q = 0; q + 1 < n; ++q) {
        double lo = bp[q], hi = bp[q + 1];
        if (hi <= lo) continue;
        double mid = 0.5 * (lo + hi), half = 0.5 * (hi - lo);
        double w1 = mid - 2.0 * r * half, w2 = mid + 2.0 * r * half;   /* mid -/+ half/sqrt(3) */
        s += half * (area2(c - g3 * w1, g1, g2) + area2(c - g3 * w2, g1, g2));
    }
    return s;
}

/* ------------------------------------------------------------------------ */
/* Wendland C2 kernel in 3D with smoothing length h_s and support 2 h_s,      */
/* written in units of h_s: W~(r) = h_s^3 W, dW~(r) = h_s^4 dW/dr.            */
/* ------------------------------------------------------------------------ */
double orc_wendland(double r)
{
    if (r >= 2.0) return 0.0;
    double e = 1.0 - 0.5 * r;
    return 21.0 / (16.0 * M_PI) * e * e * e * e * (1.0 + 2.0 * r);
}

double orc_wendland_dr(double r)
{
    if (r >= 2.0) return 0.0;
    double e = 1.0 - 0.5 * r;
    return -105.0 / (16.0 * M_PI) * r * e * e * e;
}

/* Offsets o in {-1..2}^3 (x fastest) whose data points lie within the kernel  */
/* support of the dual-cell query point: |o - (1/2,1/2,1/2)| < 2.  Returns the */
/* count and writes the offsets.                                              */
int32_t orc_support_offsets(int32_t *off /* [64][3] */)
{
    int n = 0;
    for (int oz = -1; oz <= 2; ++oz)
        for (int oy = -1; oy <= 2; ++oy)
            for (int ox = -1; ox <= 2; ++ox) {
                double rx = ox - 0.5, ry = oy - 0.5, rz = oz - 0.5;
                if (rx * rx + ry * ry + rz * rz < 4.0) {
                    off[3 * n] = ox; off[3 * n + 1] = oy; off[3 * n + 2] = oz; ++n;
                }
            }
    return n;
}

/* ------------------------------------------------------------------------ */
/* Near-surface kernel integrals at data points (fine linear indices `pts`):  */
/* query q = x_p + (h/2)(1,1,1); for each data point j within the support,    */
/* g_j is the central difference of phi at j, V_j the plane-cube fraction of  */
/* j's cell on the phi > 0 side of phi_j + g_j.(y - x_j), and                 */
/*   out[0]   = h^3 sum_j W(|q - x_j|) V_j                                     */
/*   out[1+a] = h * h^3 sum_j dW/dr(|q - x_j|) (q - x_j)_a / |q - x_j| V_j.    */
/* With h_s = h these are dimensionless and use the unit-h kernel forms.      */
/* ------------------------------------------------------------------------ */
void orc_integrals(int32_t N, double h, double B, const double *phi,
                   const int64_t *pts, int64_t n, double *out /* [n][4] */)
{
    int32_t off[64 * 3];
    const int nj = orc_support_offsets(off);
#pragma omp parallel for schedule(static)
    for (int64_t q = 0; q < n; ++q) {
        int64_t l = pts[q];
        int64_t i = l % N, j = (l / N) % N, k = l / ((int64_t)N * N);
        double kw = 0, kg[3] = {0, 0, 0};
        for (int s = 0; s < nj; ++s) {
            int64_t x = i + off[3 * s], y = j + off[3 * s + 1], z = k + off[3 * s + 2];
            double pj = rd(phi, N, x, y, z, B);
            double gx = (rd(phi, N, x + 1, y, z, B) - rd(phi, N, x - 1, y, z, B)) / (2.0 * h);
            double gy = (rd(phi, N, x, y + 1, z, B) - rd(phi, N, x, y - 1, z, B)) / (2.0 * h);
            double gz = (rd(phi, N, x, y, z + 1, B) - rd(phi, N, x, y, z - 1, B)) / (2.0 * h);
            double V = orc_plane_cube_fraction(pj / h, gx, gy, gz);
            double d[3] = {0.5 - off[3 * s], 0.5 - off[3 * s + 1], 0.5 - off[3 * s + 2]};
            double r = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
            kw += orc_wendland(r) * V;
            double dw = orc_wendland_dr(r);
            for (int a = 0; a < 3; ++a) kg[a] += dw * d[a] / r * V;
        }
        out[4 * q] = kw;
        out[4 * q + 1] = kg[0];
        out[4 * q + 2] = kg[1];
        out[4 * q + 3] = kg[2];
    }
}

/* Gather the 6x6x6 window of phi / h around data points (offsets -2..3 per    */
/* axis, x fastest): the surrogate network's input.                           */
void orc_windows(int32_t N, double h, double B, const double *phi,
                 const int64_t *pts, int64_t n, double *win /* [n][216] */)
{
#pragma omp parallel for schedule(static)
    for (int64_t q = 0; q < n; ++q) {
        int64_t l = pts[q];
        int64_t i = l % N, j = (l / N) % N, k = l / ((int64_t)N * N);
        int w = 0;
        for (int oz = -2; oz <= 3; ++oz)
            for (int oy = -2; oy <= 3; ++oy)
                for (int ox = -2; ox <= 3; ++ox)
                    win[216 * q + (w++)] = rd(phi, N, i + ox, j + oy, k + oz, B) / h;
    }
}

/* ------------------------------------------------------------------------ */
/* Surrogate MLP 216 -> 128 -> 128 -> 4 with tanh-approximated GELU.          */
/* Packed parameters: W1[128][216], b1[128], W2[128][128], b2[128],           */
/* W3[4][128], b3[4] (44,804 values).                                         */
/* ------------------------------------------------------------------------ */
enum { D_IN = 216, D_H = 128, D_OUT = 4 };
enum { O_W1 = 0, O_B1 = O_W1 + D_H * D_IN, O_W2 = O_B1 + D_H, O_B2 = O_W2 + D_H * D_H,
       O_W3 = O_B2 + D_H, O_B3 = O_W3 + D_OUT * D_H, N_PARAM = O_B3 + D_OUT };

int32_t orc_mlp_n_params(void) { return N_PARAM; }

static const double GELU_K = 0.7978845608028654;   /* sqrt(2/pi) */
static const double GELU_C = 0.044715;

double orc_gelu(double z)
{
    return 0.5 * z * (1.0 + tanh(GELU_K * (z + GELU_C * z * z * z)));
}

double orc_gelu_grad(double z)
{
    double u = GELU_K * (z + GELU_C * z * z * z);
    double th = tanh(u);
    return 0.5 * (1.0 + th) + 0.5 * z * (1.0 - th * th) * GELU_K * (1.0 + 3.0 * GELU_C * z * z);
}

static void mlp_sample(const double *w, const double *x, double *z1, double *a1,
                       double *z2, double *a2, double *y)
{
    for (int o = 0; o < D_H; ++o) {
        double s = w[O_B1 + o];
        for (int i = 0; i < D_IN; ++i) s += w[O_W1 + o * D_IN + i] * x[i];
        z1[o] = s; a1[o] = orc_gelu(s);
    }
    for (int o = 0; o < D_H; ++o) {
        double s = w[O_B2 + o];
        for (int i = 0; i < D_H; ++i) s += w[O_W2 + o * D_H + i] * a1[i];
        z2[o] = s; a2[o] = orc_gelu(s);
    }
    for (int o = 0; o < D_OUT; ++o) {
        double s = w[O_B3 + o];
        for (int i = 0; i < D_H; ++i) s += w[O_W3 + o * D_H + i] * a2[i];
        y[o] = s;
    }
}

void orc_mlp_forward(const double *w, const double *x, int64_t n, double *y)
{
#pragma omp parallel for schedule(static)
    for (int64_t q = 0; q < n; ++q) {
        double z1[D_H], a1[D_H], z2[D_H], a2[D_H];
        mlp_sample(w, x + q * D_IN, z1, a1, z2, a2, y + q * D_OUT);
    }
}

/* Gradient of sum_q dy[q] . y[q] with respect to the packed parameters      */
/* (chain rule through each layer); dw is overwritten.                        */
void orc_mlp_backward(const double *w, const double *x, const double *dy, int64_t n, double *dw)
{
    memset(dw, 0, sizeof(double) * N_PARAM);
    for (int64_t q = 0; q < n; ++q) {
        const double *xq = x + q * D_IN, *gq = dy + q * D_OUT;
        double z1[D_H], a1[D_H], z2[D_H], a2[D_H], y[D_OUT], d2[D_H], d1[D_H];
        mlp_sample(w, xq, z1, a1, z2, a2, y);
        for (int o = 0; o < D_OUT; ++o) {
            dw[O_B3 + o] += gq[o];
            for (int i = 0; i < D_H; ++i) dw[O_W3 + o * D_H + i] += gq[o] * a2[i];
        }
        for (int i = 0; i < D_H; ++i) {
            double s = 0;
            for (int o = 0; o < D_OUT; ++o) s += w[O_W3 + o * D_H + i] * gq[o];
            d2[i] = s * orc_gelu_grad(z2[i]);
        }
        for (int o = 0; o < D_H; ++o) {
            dw[O_B2 + o] += d2[o];
            for (int i = 0; i < D_H; ++i) dw[O_W2 + o * D_H + i] += d2[o] * a1[i];
        }
        for (int i = 0; i < D_H; ++i) {
            double s = 0;
            for (int o = 0; o < D_H; ++o) s += w[O_W2 + o * D_H + i] * d2[o];
            d1[i] = s * orc_gelu_grad(z1[i]);
        }
        for (int o = 0; o < D_H; ++o) {
            dw[O_B1 + o] += d1[o];
            for (int i = 0; i < D_IN; ++i) dw[O_W1 + o * D_IN + i] += d1[o] * xq[i];
        }
    }
}

/* Adam (Kingma & Ba, 2015), step t >= 1, bias-corrected moments.            */
void orc_adam(int64_t n, double *w, const double *g, double *m, double *v, int64_t t,
              double lr, double beta1, double beta2, double eps)
{
    double c1 = 1.0 - pow(beta1, (double)t), c2 = 1.0 - pow(beta2, (double)t);
    for (int64_t i = 0; i < n; ++i) {
        m[i] = beta1 * m[i] + (1.0 - beta1) * g[i];
        v[i] = beta2 * v[i] + (1.0 - beta2) * g[i] * g[i];
        double mh = m[i] / c1, vh = v[i] / c2;
        w[i] -= lr * mh / (sqrt(vh) + eps);
    }
}
