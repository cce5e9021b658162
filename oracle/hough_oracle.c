/*
 * hough_oracle.c -- plain, slow CPU oracle of the fixed-point Hough transform.
 *
 * TEST INFRASTRUCTURE, NOT PRODUCT CODE.  Only the test-suite, the smoke check
 * and the benchmark's CPU-baseline leg load this library.  It shares no code,
 * header, table or constant generator with the GPU library: every constant is
 * derived here from its definition, every value is recomputed per sample.
 *
 * What it computes (Halyo et al., "GPU Enhancement of the Trigger to Extend
 * Physics Reach at the LHC", Sec. "Proposed Fast Tracking Algorithm" and its
 * Fig. "hough" caption; Sec. "Preliminary Results", the curved-track and
 * displaced-track paragraph):
 *   - every hit is mapped to the set of helix parameters it is compatible
 *     with; votes of all hits are summed in a binned parameter space;
 *   - local maxima of that space are the track candidates;
 *   - the hits that voted for a candidate are the input of the track fit
 *     (Sec. "Preliminary Results", fitting paragraph);
 *   - a second transform of the candidates themselves finds the vertices of
 *     displaced jets (Sec. "New Trigger Capabilities");
 *   - for the paper's own detector (x/y smear), a variant of the transform
 *     with each hit's own radius and an integer arcsine.
 * The paper gives no parameterisation, grid, binning or tie rule.  The
 * discretisation used here is the "fixed-point transform" written out step by
 * step below (one reading of the silent points; the same reading is stated in
 * the design notes of the repository).
 *
 * Parameters: phi0 (azimuth of the track direction at the point of closest
 * approach, PCA), q/pT (GeV^-1) and d0 (signed transverse impact parameter,
 * cm; PCA = d0 * (-sin phi0, cos phi0)).  Signed curvature c = -kappa * q/pT
 * with kappa = 0.299792458e-2 * B (B in tesla, lengths in cm): positive charges
 * bend clockwise for B along +z.  A point at radius r on the circle, on the
 * branch leaving the PCA, has azimuth phi with
 *     sin(phi - phi0) = A(r, c, d0) = (c (r^2 + d0^2) + 2 d0) / (2 r (1 + c d0)),
 * so phi0 = phi - asin(A).  For d0 = 0 this is phi0 = phi - asin(c r / 2).
 *
 * Parity status of each function: see the pins in tests/test_oracle_pins.py.
 * All functions here are pinned; none is "parity unpinned".
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif

/* Configuration as plain numbers (the oracle's own struct). */
typedef struct {
    int32_t n_layers;
    const double* r_cm;        /* nominal layer radii */
    const double* halflen_cm;  /* may be NULL; not used by the transform */
    double B_tesla;
    int32_t n_phi, n_qpt, n_d0;
    int32_t frac_bits;         /* F: angle bits below one phi0 bin */
    double qpt_min, qpt_max, d0_min, d0_max;
    int32_t n_cot, n_z0;
    double cot_min, cot_max, z0_min, z0_max;
} or_cfg_t;

/* ------------------------------------------------------------------------ */
/* Step 1 of the transform: Q16.16 fixed point of a float coordinate.        */
/* The float is scaled by 2^16 (exact) and rounded to nearest, ties to even. */
/* ------------------------------------------------------------------------ */
int32_t or_q16(float v)
{
    double s = (double)v * 65536.0;
    return (int32_t)llrint(s);
}

/* A coordinate is usable when it is finite and strictly inside +-32768 cm. */
static int or_coord_ok(float v)
{
    return isfinite(v) && fabsf(v) < 32768.0f;
}

/* ------------------------------------------------------------------------ */
/* Step 2: azimuth of (X, Y) in 32-bit binary angle measure (2^32 == 2 pi),  */
/* by integer CORDIC in vectoring mode (Volder, 1959).                       */
/*   - turn the vector by -90 degrees until it lies in [0, 90) degrees,      */
/*     counting the quarter turns q;                                         */
/*   - 16 guard bits; 30 micro-rotations by atan(2^-i), each pushing y       */
/*     towards zero, accumulating the signed angle constants                 */
/*     T_i = round(atan(2^-i) * 2^31 / pi);                                  */
/*   - result = q * 2^30 + accumulated angle, modulo 2^32.                   */
/* ------------------------------------------------------------------------ */
static int64_t or_cordic_const(int i)
{
    return llrint(atan(ldexp(1.0, -i)) * (2147483648.0 / M_PI));
}

uint32_t or_azimuth(int32_t X, int32_t Y)
{
    int64_t x = X, y = Y, tmp, dx, dy, theta = 0;
    uint32_t quarter = 0;
    int i;
    while (!(x > 0 && y >= 0)) { /* rotate by -90 degrees */
        tmp = x;
        x = y;
        y = -tmp;
        quarter++;
    }
    x *= 65536;
    y *= 65536;
    for (i = 0; i < 30; i++) {
        dx = x >> i; /* arithmetic shifts (floor) */
        dy = y >> i;
        if (y >= 0) {
            x = x + dy;
            y = y - dx;
            theta += or_cordic_const(i);
        } else {
            x = x - dy;
            y = y + dx;
            theta -= or_cordic_const(i);
        }
    }
    return (uint32_t)((uint64_t)quarter * 1073741824ull + (uint64_t)theta);
}

/* Validity of one hit and its fixed-point coordinates. */
int or_hit(float x, float y, uint8_t layer, int32_t n_layers, int32_t* X, int32_t* Y)
{
    if ((int32_t)layer >= n_layers) return 0;
    if (!or_coord_ok(x) || !or_coord_ok(y)) return 0;
    *X = or_q16(x);
    *Y = or_q16(y);
    if (*X == 0 && *Y == 0) return 0;
    return 1;
}

/* Per-hit preparation for a batch: azimuth (32-bit BAM) and validity. */
void or_prep(int32_t n, const float* x, const float* y, const uint8_t* layer, int32_t n_layers,
             uint32_t* phi_out, uint8_t* valid_out)
{
    int32_t h, X, Y;
    for (h = 0; h < n; h++) {
        valid_out[h] = (uint8_t)or_hit(x[h], y[h], layer[h], n_layers, &X, &Y);
        phi_out[h] = valid_out[h] ? or_azimuth(X, Y) : 0u;
    }
}

/* ------------------------------------------------------------------------ */
/* Step 3: grid.  Bin centres of q/pT and d0; phi0 bins are the top          */
/* log2(n_phi) bits of an M-bit angle, M = log2(n_phi) + F.                  */
/* ------------------------------------------------------------------------ */
static int or_log2(int32_t v)
{
    int s = 0;
    while ((1 << s) < v) s++;
    return s;
}

int32_t or_angle_bits(const or_cfg_t* g)
{
    return or_log2(g->n_phi) + g->frac_bits;
}

double or_qpt_centre(const or_cfg_t* g, int32_t k)
{
    return g->qpt_min + ((double)k + 0.5) * ((g->qpt_max - g->qpt_min) / (double)g->n_qpt);
}

double or_d0_centre(const or_cfg_t* g, int32_t l)
{
    return g->d0_min + ((double)l + 0.5) * ((g->d0_max - g->d0_min) / (double)g->n_d0);
}

double or_curvature(const or_cfg_t* g, int32_t k)
{
    double kappa = 0.299792458e-2 * g->B_tesla;
    return -kappa * or_qpt_centre(g, k);
}

/* ------------------------------------------------------------------------ */
/* Step 4: one sample.  For a hit on a layer of radius r and the parameter   */
/* cell (c, d), the phi0 offset asin(A) in M-bit BAM, or "invalid" when the  */
/* circle does not reach radius r (|A| > 1) or the denominator is not        */
/* positive.  Evaluated per call, in IEEE double, in this operation order.   */
/* ------------------------------------------------------------------------ */
int or_sample(double r, double c, double d, int32_t M, int32_t* E)
{
    double num = c * (r * r + d * d) + 2.0 * d;
    double den = 2.0 * r * (1.0 + c * d);
    double A, K;
    if (!(den > 0.0)) return 0;
    A = num / den;
    if (!(fabs(A) <= 1.0)) return 0;
    K = ldexp(1.0, M - 1) / M_PI;
    *E = (int32_t)llrint(asin(A) * K);
    return 1;
}

/* phi0 bin of a hit with M-bit azimuth phiM for sample value E. */
static int32_t or_bin(uint32_t phiM, int32_t E, int32_t M, int32_t F)
{
    uint32_t mask = (M >= 32) ? 0xffffffffu : ((1u << M) - 1u);
    return (int32_t)(((phiM - (uint32_t)E) & mask) >> F);
}

/* ------------------------------------------------------------------------ */
/* Step 5: vote.  acc[l][k][b] (b fastest), int32, fully overwritten.        */
/* For every valid hit, every d0 bin l and every q/pT bin k whose sample is  */
/* valid: one vote into the phi0 bin of phi - asin(A).                       */
/* Returns the number of votes cast.                                         */
/* ------------------------------------------------------------------------ */
int64_t or_vote(const or_cfg_t* g, int32_t n, const float* x, const float* y, const uint8_t* layer,
                int32_t* acc)
{
    int32_t M = or_angle_bits(g), F = g->frac_bits;
    int64_t total = 0, nbins = (int64_t)g->n_d0 * g->n_qpt * g->n_phi;
    uint32_t* phiM = (uint32_t*)malloc(sizeof(uint32_t) * (size_t)(n > 0 ? n : 1));
    uint8_t* ok = (uint8_t*)malloc((size_t)(n > 0 ? n : 1));
    int32_t h, l;
    or_prep(n, x, y, layer, g->n_layers, phiM, ok);
    for (h = 0; h < n; h++) phiM[h] >>= (32 - M);
    memset(acc, 0, sizeof(int32_t) * (size_t)nbins);
#pragma omp parallel for schedule(dynamic, 1) reduction(+ : total)
    for (l = 0; l < g->n_d0; l++) {
        double d = or_d0_centre(g, l);
        int32_t hh, k, E;
        for (hh = 0; hh < n; hh++) {
            if (!ok[hh]) continue;
            for (k = 0; k < g->n_qpt; k++) {
                double c = or_curvature(g, k);
                if (!or_sample(g->r_cm[layer[hh]], c, d, M, &E)) continue;
                acc[((int64_t)l * g->n_qpt + k) * g->n_phi + or_bin(phiM[hh], E, M, F)] += 1;
                total += 1;
            }
        }
    }
    free(phiM);
    free(ok);
    return total;
}

/* The same votes restricted to a list of (l, k) columns: out[i][b] for the  */
/* column (cols[2i], cols[2i+1]).  Used to check large accumulators by       */
/* sampling columns.                                                          */
void or_vote_columns(const or_cfg_t* g, int32_t n, const float* x, const float* y,
                     const uint8_t* layer, int32_t n_cols, const int32_t* cols, int32_t* out)
{
    int32_t M = or_angle_bits(g), F = g->frac_bits;
    uint32_t* phiM = (uint32_t*)malloc(sizeof(uint32_t) * (size_t)(n > 0 ? n : 1));
    uint8_t* ok = (uint8_t*)malloc((size_t)(n > 0 ? n : 1));
    int32_t h, i;
    or_prep(n, x, y, layer, g->n_layers, phiM, ok);
    for (h = 0; h < n; h++) phiM[h] >>= (32 - M);
    memset(out, 0, sizeof(int32_t) * (size_t)n_cols * g->n_phi);
#pragma omp parallel for schedule(dynamic, 1)
    for (i = 0; i < n_cols; i++) {
        int32_t l = cols[2 * i], k = cols[2 * i + 1], hh, E;
        double d = or_d0_centre(g, l), c = or_curvature(g, k);
        for (hh = 0; hh < n; hh++) {
            if (!ok[hh]) continue;
            if (!or_sample(g->r_cm[layer[hh]], c, d, M, &E)) continue;
            out[(int64_t)i * g->n_phi + or_bin(phiM[hh], E, M, F)] += 1;
        }
    }
    free(phiM);
    free(ok);
}

/* ------------------------------------------------------------------------ */
/* Step 6: peaks.  Bin i = (l, k, b) is a candidate iff acc[i] >= thr and,   */
/* for every neighbour j in the 3x3x3 block around it (phi0 cyclic, q/pT and */
/* d0 clipped at the grid edge), acc[i] > acc[j] when j precedes i and       */
/* acc[i] >= acc[j] otherwise.  j precedes i when (l_j, k_j) < (l_i, k_i)    */
/* lexicographically, or when j is the previous phi0 bin (b - 1 mod n_phi)   */
/* of the same (l, k) column.  Output in increasing linear index            */
/* (l * n_qpt + k) * n_phi + b as {l, k, b, votes}; only the first `cap` are */
/* written; the return value is the total count.                             */
/* ------------------------------------------------------------------------ */
static int or_is_peak(const or_cfg_t* g, const int32_t* acc, int32_t l, int32_t k, int32_t b, int32_t thr)
{
    int32_t Nd = g->n_d0, Nk = g->n_qpt, Np = g->n_phi, dl, dk, db;
    int32_t v = acc[((int64_t)l * Nk + k) * Np + b];
    if (v < thr) return 0;
    for (dl = -1; dl <= 1; dl++) {
        int32_t l2 = l + dl;
        if (l2 < 0 || l2 >= Nd) continue;
        for (dk = -1; dk <= 1; dk++) {
            int32_t k2 = k + dk;
            if (k2 < 0 || k2 >= Nk) continue;
            for (db = -1; db <= 1; db++) {
                int32_t b2, u, precedes;
                if (dl == 0 && dk == 0 && db == 0) continue;
                b2 = (b + db + Np) % Np;
                u = acc[((int64_t)l2 * Nk + k2) * Np + b2];
                precedes = (l2 < l) || (l2 == l && k2 < k) || (l2 == l && k2 == k && db == -1);
                if (precedes ? !(v > u) : !(v >= u)) return 0;
            }
        }
    }
    return 1;
}

int64_t or_peaks(const or_cfg_t* g, const int32_t* acc, int32_t thr, int64_t cap, int32_t* out)
{
    int64_t count = 0;
    int32_t l, k, b;
    for (l = 0; l < g->n_d0; l++)
        for (k = 0; k < g->n_qpt; k++)
            for (b = 0; b < g->n_phi; b++) {
                if (!or_is_peak(g, acc, l, k, b, thr)) continue;
                if (count < cap) {
                    out[4 * count + 0] = l;
                    out[4 * count + 1] = k;
                    out[4 * count + 2] = b;
                    out[4 * count + 3] = acc[((int64_t)l * g->n_qpt + k) * g->n_phi + b];
                }
                count++;
            }
    return count;
}

/* Peak test of a single bin (for sampled checks of large accumulators). */
int or_peak_at(const or_cfg_t* g, const int32_t* acc, int32_t l, int32_t k, int32_t b, int32_t thr)
{
    return or_is_peak(g, acc, l, k, b, thr);
}

/* ------------------------------------------------------------------------ */
/* Step 7: assignment.  For each candidate p = (l_p, k_p, b_p), the valid    */
/* hits whose sample at (l_p, k_p) is valid and falls in phi0 bin b_p (so    */
/* the list length equals acc at the candidate).  Order: layer by layer from */
/* the innermost layer outwards, within a layer by the hit's angle inside    */
/* the bin, rel = ((PhiM - E) mod 2^M) - b_p * 2^F, ties by hit index -- the */
/* order in which a track fit meets the hits along the track.               */
/* CSR output: offsets[0..n_peaks], hit_idx[offsets[p] .. offsets[p+1]),    */
/* entries at positions >= cap_pairs are not written.  Returns the total.    */
/* The sample values of the candidate's cell are evaluated once per layer    */
/* for each candidate (they depend only on the layer, l_p and k_p).          */
/* ------------------------------------------------------------------------ */
typedef struct {
    uint32_t rel;
    int32_t h;
} or_member_t;

static int or_member_cmp(const void* a, const void* b)
{
    const or_member_t* x = (const or_member_t*)a;
    const or_member_t* y = (const or_member_t*)b;
    if (x->rel != y->rel) return x->rel < y->rel ? -1 : 1;
    return (x->h > y->h) - (x->h < y->h);
}

int64_t or_assign(const or_cfg_t* g, int32_t n, const float* x, const float* y, const uint8_t* layer,
                  int32_t n_peaks, const int32_t* peaks, int64_t* offsets, int32_t* hit_idx,
                  int64_t cap_pairs)
{
    int32_t M = or_angle_bits(g), F = g->frac_bits, p, h, L, i, m;
    uint32_t mask = (M >= 32) ? 0xffffffffu : ((1u << M) - 1u);
    uint32_t* phiM = (uint32_t*)malloc(sizeof(uint32_t) * (size_t)(n > 0 ? n : 1));
    uint8_t* ok = (uint8_t*)malloc((size_t)(n > 0 ? n : 1));
    or_member_t* mem = (or_member_t*)malloc(sizeof(or_member_t) * (size_t)(n > 0 ? n : 1));
    int64_t pos = 0;
    or_prep(n, x, y, layer, g->n_layers, phiM, ok);
    for (h = 0; h < n; h++) phiM[h] >>= (32 - M);
    for (p = 0; p < n_peaks; p++) {
        int32_t lp = peaks[4 * p], kp = peaks[4 * p + 1], bp = peaks[4 * p + 2];
        double d = or_d0_centre(g, lp), c = or_curvature(g, kp);
        offsets[p] = pos;
        for (L = 0; L < g->n_layers; L++) {
            int32_t E;
            if (!or_sample(g->r_cm[L], c, d, M, &E)) continue;
            m = 0;
            for (h = 0; h < n; h++) {
                if (!ok[h] || layer[h] != L) continue;
                if (or_bin(phiM[h], E, M, F) != bp) continue;
                mem[m].rel = ((phiM[h] - (uint32_t)E) & mask) - ((uint32_t)bp << F);
                mem[m].h = h;
                m++;
            }
            qsort(mem, (size_t)m, sizeof(or_member_t), or_member_cmp);
            for (i = 0; i < m; i++) {
                if (pos < cap_pairs) hit_idx[pos] = mem[i].h;
                pos++;
            }
        }
    }
    offsets[n_peaks] = pos;
    free(phiM);
    free(ok);
    free(mem);
    return pos;
}

/* ------------------------------------------------------------------------ */
/* Step 8 (second stage, r-z): for one candidate (l, k), vote its hits into  */
/* a cot(theta) x z0 grid with the helix model z = z0 + s cot(theta), where  */
/* s is the transverse arc length from the PCA to the hit:                    */
/*   chord  Lc = sqrt(r^2 + d^2 - 2 d r A),                                   */
/*   arc    s  = Lc                    if c == 0,                             */
/*             = (2/|c|) asin(|c| Lc/2) otherwise;                            */
/* S = round(s * 2^16) (Q16.16), C_m = round(cot_m * 2^16) at the bin centre, */
/* z0 = Z * 2^16 - S * C_m exactly in Q32.32; bin j = floor((z0 - z0min)/W)  */
/* with z0min = round(z0_min * 2^32) and W = round(bin width * 2^32).        */
/* Output per candidate: the bin with most votes (lowest m * n_z0 + j among  */
/* ties) and its count, or (-1, -1, 0) when nothing voted.                    */
/* ------------------------------------------------------------------------ */
int or_arclen(double r, double c, double d, int64_t* S)
{
    double num = c * (r * r + d * d) + 2.0 * d;
    double den = 2.0 * r * (1.0 + c * d);
    double A, Lc2, Lc, s, u;
    if (!(den > 0.0)) return 0;
    A = num / den;
    if (!(fabs(A) <= 1.0)) return 0;
    Lc2 = r * r + d * d - 2.0 * d * r * A;
    Lc = sqrt(Lc2 > 0.0 ? Lc2 : 0.0);
    if (c == 0.0) {
        s = Lc;
    } else {
        u = fabs(c) * Lc / 2.0;
        if (u > 1.0) u = 1.0;
        s = (2.0 / fabs(c)) * asin(u);
    }
    *S = llrint(s * 65536.0);
    return 1;
}

int64_t or_cot_centre_q16(const or_cfg_t* g, int32_t m)
{
    double v = g->cot_min + ((double)m + 0.5) * ((g->cot_max - g->cot_min) / (double)g->n_cot);
    return llrint(v * 65536.0);
}

void or_zvote(const or_cfg_t* g, int32_t n, const float* z, const uint8_t* layer, int32_t n_peaks,
              const int32_t* peaks, const int64_t* offsets, const int32_t* hit_idx, int32_t* out)
{
    int64_t z0min = llrint(g->z0_min * 4294967296.0);
    int64_t W = llrint(((g->z0_max - g->z0_min) / (double)g->n_z0) * 4294967296.0);
    int32_t* zacc = (int32_t*)malloc(sizeof(int32_t) * (size_t)g->n_cot * g->n_z0);
    int64_t* C = (int64_t*)malloc(sizeof(int64_t) * (size_t)g->n_cot);
    int32_t p, m;
    (void)n;
    for (m = 0; m < g->n_cot; m++) C[m] = or_cot_centre_q16(g, m);
    for (p = 0; p < n_peaks; p++) {
        int32_t lp = peaks[4 * p], kp = peaks[4 * p + 1], best = -1, bestv = 0, i;
        double d = or_d0_centre(g, lp), c = or_curvature(g, kp);
        int64_t q;
        memset(zacc, 0, sizeof(int32_t) * (size_t)g->n_cot * g->n_z0);
        for (q = offsets[p]; q < offsets[p + 1]; q++) {
            int32_t h = hit_idx[q], Z;
            int64_t S;
            if (!or_coord_ok(z[h])) continue;
            Z = or_q16(z[h]);
            if (!or_arclen(g->r_cm[layer[h]], c, d, &S)) continue;
            for (m = 0; m < g->n_cot; m++) {
                int64_t z0 = (int64_t)Z * 65536 - S * C[m] - z0min;
                int64_t j;
                if (z0 < 0) continue;
                j = z0 / W;
                if (j >= g->n_z0) continue;
                zacc[(int64_t)m * g->n_z0 + j] += 1;
            }
        }
        for (i = 0; i < g->n_cot * g->n_z0; i++)
            if (zacc[i] > bestv) {
                bestv = zacc[i];
                best = i;
            }
        out[3 * p + 0] = best < 0 ? -1 : best / g->n_z0;
        out[3 * p + 1] = best < 0 ? -1 : best % g->n_z0;
        out[3 * p + 2] = bestv;
    }
    free(zacc);
    free(C);
}

/* Track fit of each candidate's hits (Sec. "Preliminary Results", fitting paragraph: the hits
 * of a candidate go on to a fit; the paper names no method).  Reading: the algebraic circle fit
 * of Kasa (I. Kasa, "A circle fitting procedure and its error analysis", IEEE Trans. Instrum.
 * Meas. 25 (1976) 8-14): the circle x^2 + y^2 + a x + b y + c = 0 minimising
 *     sum_i (x_i^2 + y_i^2 + a x_i + b y_i + c)^2,
 * i.e. the 3x3 normal equations
 *     | Sxx Sxy Sx | |a|     | Sxz |
 *     | Sxy Syy Sy | |b| = - | Syz |      (z = x^2 + y^2, S = sum over the hits)
 *     | Sx  Sy  N  | |c|     | Sz  |
 * solved by Cramer's rule; centre (-a/2, -b/2), R^2 = xc^2 + yc^2 - c.  The sums run over the
 * candidate's hit list in its order, hits in cm (float32 converted to double).  Fewer than 3 hits
 * or a zero determinant: centre (0, 0), R^2 = -1.  out[4 p .. 4 p + 3] = xc, yc, R^2, N. */
void or_fit(const float* x, const float* y, int32_t n_peaks, const int64_t* offsets, const int32_t* hit_idx,
            double* out)
{
    int32_t p;
    for (p = 0; p < n_peaks; p++) {
        double sx = 0.0, sy = 0.0, sxx = 0.0, sxy = 0.0, syy = 0.0, sz = 0.0, sxz = 0.0, syz = 0.0;
        double N, det, r0, r1, r2, a, b, c, xc, yc;
        int64_t q;
        for (q = offsets[p]; q < offsets[p + 1]; q++) {
            double X = (double)x[hit_idx[q]], Y = (double)y[hit_idx[q]];
            double Z = X * X + Y * Y;
            sx += X;
            sy += Y;
            sxx += X * X;
            sxy += X * Y;
            syy += Y * Y;
            sz += Z;
            sxz += X * Z;
            syz += Y * Z;
        }
        N = (double)(offsets[p + 1] - offsets[p]);
        det = sxx * (syy * N - sy * sy) - sxy * (sxy * N - sy * sx) + sx * (sxy * sy - syy * sx);
        out[4 * p + 3] = N;
        if (N < 3.0 || det == 0.0) {
            out[4 * p + 0] = 0.0;
            out[4 * p + 1] = 0.0;
            out[4 * p + 2] = -1.0;
            continue;
        }
        r0 = -sxz;
        r1 = -syz;
        r2 = -sz;
        a = (r0 * (syy * N - sy * sy) - sxy * (r1 * N - sy * r2) + sx * (r1 * sy - syy * r2)) / det;
        b = (sxx * (r1 * N - r2 * sy) - r0 * (sxy * N - sy * sx) + sx * (sxy * r2 - r1 * sx)) / det;
        c = (sxx * (syy * r2 - sy * r1) - sxy * (sxy * r2 - r1 * sx) + r0 * (sxy * sy - syy * sx)) / det;
        xc = -a / 2.0;
        yc = -b / 2.0;
        out[4 * p + 0] = xc;
        out[4 * p + 1] = yc;
        out[4 * p + 2] = xc * xc + yc * yc - c;
    }
}

/* ------------------------------------------------------------------------ */
/* Step 10 (second Hough transform, Sec. "New Trigger Capabilities" and its  */
/* displaced-jet figures): the candidates of the first transform are the    */
/* input; tracks from one displaced vertex are candidates whose curves all   */
/* pass through that vertex, so each candidate votes for every vertex        */
/* position its own helix passes through, and local maxima of that vertex    */
/* space are the vertices.                                                   */
/*   Vertex space: radius rows j, centres r_j = r_min + (j + 0.5) *          */
/*   ((r_max - r_min) / n_vr), times n_vphi azimuth bins (a power of two);   */
/*   an azimuth bin holds 2^(M - log2 n_vphi) values of the first           */
/*   transform's M-bit angle.                                                */
/*   A candidate (l, k, b) stands for the helix of its bin centres: d0 and   */
/*   q/pT centres of l and k, and phi0 = the centre of bin b, the M-bit      */
/*   angle b * 2^F + 2^(F-1).  On the branch leaving its PCA the helix meets */
/*   radius r_j at azimuth phi0 + asin(A(r_j, c, d0)) (step 4 solved for phi */
/*   instead of phi0), so with E_j = the step-4 sample at radius r_j:        */
/*       vertex azimuth (M-bit) = (phi0 + E_j) mod 2^M,                      */
/*       bin = that >> (M - log2 n_vphi).                                    */
/*   One vote per row whose sample is valid, for every candidate with at     */
/*   least min_votes first-stage votes.  acc_v[j][bin] (bin fastest), fully   */
/*   overwritten.  Returns the number of votes cast.                         */
/* Vertex peaks are step 6 on the grid (1 x n_vr x n_vphi): radius rows take */
/* the place of q/pT rows (clipped), azimuth that of phi0 (cyclic).          */
/* ------------------------------------------------------------------------ */
double or_vertex_radius(int32_t n_vr, double r_min, double r_max, int32_t j)
{
    return r_min + ((double)j + 0.5) * ((r_max - r_min) / (double)n_vr);
}

int64_t or_vertex_vote(const or_cfg_t* g, int32_t n_vr, int32_t n_vphi, double r_min, double r_max,
                       int32_t min_votes, int32_t n_peaks, const int32_t* pk, int32_t* acc_v)
{
    int32_t M = or_angle_bits(g), F = g->frac_bits, lv = or_log2(n_vphi), p, j;
    uint32_t mask = (M >= 32) ? 0xffffffffu : ((1u << M) - 1u);
    int64_t votes = 0;
    memset(acc_v, 0, sizeof(int32_t) * (size_t)n_vr * (size_t)n_vphi);
    for (p = 0; p < n_peaks; p++) {
        int32_t l = pk[4 * p + 0], k = pk[4 * p + 1], b = pk[4 * p + 2];
        double c, d;
        uint32_t phi0;
        if (pk[4 * p + 3] < min_votes) continue;
        c = or_curvature(g, k);
        d = or_d0_centre(g, l);
        phi0 = ((uint32_t)b << F) + (1u << (F - 1));
        for (j = 0; j < n_vr; j++) {
            int32_t E;
            uint32_t v;
            if (!or_sample(or_vertex_radius(n_vr, r_min, r_max, j), c, d, M, &E)) continue;
            v = (phi0 + (uint32_t)E) & mask;
            acc_v[(int64_t)j * n_vphi + (int32_t)(v >> (M - lv))]++;
            votes++;
        }
    }
    return votes;
}

/* ------------------------------------------------------------------------ */
/* Step 11 (per-hit radius, the paper's detector with its x/y smear): the    */
/* transform of step 4-5 with each hit's own radius instead of its layer's,  */
/* and the arcsine taken in integers so that any two implementations agree: */
/*   R  = floor(sqrt(X^2 + Y^2)) in Q16.16 (exact integer square root),      */
/*        r = R / 2^16;                                                      */
/*   A  as in step 4 (IEEE double, same operation order, same validity);     */
/*   a  = llrint(A * 2^30) (Q2.30), b = floor(sqrt(2^60 - a^2)),             */
/*   t  = the step-2 CORDIC angle of the vector (b, a), read as a signed      */
/*        32-bit binary angle (= asin(A), |t| <= 2^30);                      */
/*   E  = floor((t + 2^(31-M)) / 2^(32-M))   (round half up to M bits).      */
/* Votes as in step 5 with this E; the layer only decides validity.         */
/* ------------------------------------------------------------------------ */
uint64_t or_isqrt(uint64_t v)
{
    /* digit-by-digit square root in base 4: exact floor(sqrt(v)) */
    uint64_t rem = v, root = 0, bit = (uint64_t)1 << 62;
    while (bit > rem) bit >>= 2;
    while (bit) {
        if (rem >= root + bit) {
            rem -= root + bit;
            root = (root >> 1) + bit;
        } else {
            root >>= 1;
        }
        bit >>= 2;
    }
    return root;
}

int or_sample_cr(double r, double c, double d, int32_t M, int32_t* E)
{
    double num = c * (r * r + d * d) + 2.0 * d;
    double den = 2.0 * r * (1.0 + c * d);
    double A;
    int64_t a, b, t;
    int32_t s = 32 - M;
    if (!(den > 0.0)) return 0;
    A = num / den;
    if (!(fabs(A) <= 1.0)) return 0;
    a = llrint(A * 1073741824.0);
    b = (int64_t)or_isqrt((uint64_t)(((int64_t)1 << 60) - a * a));
    t = (int64_t)(int32_t)or_azimuth((int32_t)b, (int32_t)a);
    *E = (int32_t)((t + ((int64_t)1 << (s - 1))) >> s);
    return 1;
}

double or_hit_radius(int32_t X, int32_t Y)
{
    uint64_t R2 = (uint64_t)((int64_t)X * X) + (uint64_t)((int64_t)Y * Y);
    return (double)or_isqrt(R2) / 65536.0;
}

int64_t or_vote_cr(const or_cfg_t* g, int32_t n, const float* x, const float* y, const uint8_t* layer,
                   int32_t* acc)
{
    int32_t M = or_angle_bits(g), F = g->frac_bits, h, l, k;
    int64_t votes = 0;
    memset(acc, 0, sizeof(int32_t) * (size_t)g->n_d0 * g->n_qpt * g->n_phi);
    for (h = 0; h < n; h++) {
        int32_t X, Y;
        uint32_t phiM;
        double r;
        if (!or_hit(x[h], y[h], layer[h], g->n_layers, &X, &Y)) continue;
        phiM = or_azimuth(X, Y) >> (32 - M);
        r = or_hit_radius(X, Y);
        for (l = 0; l < g->n_d0; l++) {
            double d = or_d0_centre(g, l);
            for (k = 0; k < g->n_qpt; k++) {
                int32_t E;
                if (!or_sample_cr(r, or_curvature(g, k), d, M, &E)) continue;
                acc[((int64_t)l * g->n_qpt + k) * g->n_phi + or_bin(phiM, E, M, F)] += 1;
                votes++;
            }
        }
    }
    return votes;
}

/* Assignment with each hit's own radius (the step-7 lists for the step-11  */
/* transform): for each candidate p = (l_p, k_p, b_p), the valid hits whose */
/* per-hit-radius sample at (l_p, k_p) is valid and falls in phi0 bin b_p   */
/* (so the list length equals the step-11 accumulator at the candidate),    */
/* in the step-7 order: layer, angle inside the bin, hit index.             */
int64_t or_assign_cr(const or_cfg_t* g, int32_t n, const float* x, const float* y, const uint8_t* layer,
                     int32_t n_peaks, const int32_t* peaks, int64_t* offsets, int32_t* hit_idx,
                     int64_t cap_pairs)
{
    int32_t M = or_angle_bits(g), F = g->frac_bits, p, h, L, i, m;
    uint32_t mask = (M >= 32) ? 0xffffffffu : ((1u << M) - 1u);
    uint32_t* phiM = (uint32_t*)malloc(sizeof(uint32_t) * (size_t)(n > 0 ? n : 1));
    double* rad = (double*)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    uint8_t* ok = (uint8_t*)malloc((size_t)(n > 0 ? n : 1));
    or_member_t* mem = (or_member_t*)malloc(sizeof(or_member_t) * (size_t)(n > 0 ? n : 1));
    int64_t pos = 0;
    for (h = 0; h < n; h++) {
        int32_t X, Y;
        ok[h] = (uint8_t)or_hit(x[h], y[h], layer[h], g->n_layers, &X, &Y);
        phiM[h] = ok[h] ? or_azimuth(X, Y) >> (32 - M) : 0u;
        rad[h] = ok[h] ? or_hit_radius(X, Y) : 0.0;
    }
    for (p = 0; p < n_peaks; p++) {
        int32_t lp = peaks[4 * p], kp = peaks[4 * p + 1], bp = peaks[4 * p + 2];
        double d = or_d0_centre(g, lp), c = or_curvature(g, kp);
        offsets[p] = pos;
        for (L = 0; L < g->n_layers; L++) {
            m = 0;
            for (h = 0; h < n; h++) {
                int32_t E;
                if (!ok[h] || layer[h] != L) continue;
                if (!or_sample_cr(rad[h], c, d, M, &E)) continue;
                if (bp != or_bin(phiM[h], E, M, F)) continue;
                mem[m].rel = ((phiM[h] - (uint32_t)E) & mask) - ((uint32_t)bp << F);
                mem[m].h = h;
                m++;
            }
            qsort(mem, (size_t)m, sizeof(or_member_t), or_member_cmp);
            for (i = 0; i < m; i++) {
                if (pos < cap_pairs) hit_idx[pos] = mem[i].h;
                pos++;
            }
        }
    }
    offsets[n_peaks] = pos;
    free(phiM);
    free(rad);
    free(ok);
    free(mem);
    return pos;
}

/* ------------------------------------------------------------------------ */
/* Background suppression inside a candidate's bin (refinement).  The hits   */
/* of a crowded bin come from the track and from other tracks crossing the   */
/* bin; the track's own hits agree on phi0 far more closely than the bin     */
/* width, at its (d0, q/pT), so they sit together in the angle inside the    */
/* bin.  For candidate p = (l, k, b) with hit list H (step 7) and each listed */
/* hit's angle inside the bin rel = ((PhiM - E) mod 2^M) - b * 2^F (E the    */
/* sample of its layer at (l, k)): among the windows [c, c + w) that begin  */
/* at a listed hit's rel, take the one holding hits of the most distinct    */
/* layers, then the most hits, then the lowest c; the refined list keeps,   */
/* for every layer present in the window, the hit nearest the window centre */
/* c + w/2 (smallest |2 rel - 2c - w|, ties by the lower hit index).         */
/* out_hits[p * n_layers + L] = that hit or -1; out_layers[p] = the number  */
/* of layers of the refined list (0 for an empty list).  Returns the total  */
/* number of refined entries.                                               */
/* ------------------------------------------------------------------------ */
int64_t or_refine(const or_cfg_t* g, int32_t n, const float* x, const float* y, const uint8_t* layer,
                  int32_t n_peaks, const int32_t* peaks, const int64_t* offsets, const int32_t* hit_idx, int32_t w,
                  int32_t* out_hits, int32_t* out_layers)
{
    int32_t M = or_angle_bits(g), F = g->frac_bits, NL = g->n_layers, p, i, j, L;
    uint32_t mask = (M >= 32) ? 0xffffffffu : ((1u << M) - 1u);
    uint32_t* phi = (uint32_t*)malloc(sizeof(uint32_t) * (size_t)(n > 0 ? n : 1));
    uint8_t* ok = (uint8_t*)malloc((size_t)(n > 0 ? n : 1));
    int64_t total = 0;
    or_prep(n, x, y, layer, NL, phi, ok);
    for (p = 0; p < n_peaks; p++) {
        int32_t lp = peaks[4 * p], kp = peaks[4 * p + 1], bp = peaks[4 * p + 2];
        double d = or_d0_centre(g, lp), c = or_curvature(g, kp);
        int64_t q0 = offsets[p], m = offsets[p + 1] - offsets[p];
        int32_t E[64], best_l = -1, best_n = -1, best_c = 0;
        int64_t* rel = (int64_t*)malloc(sizeof(int64_t) * (size_t)(m > 0 ? m : 1));
        for (L = 0; L < NL; L++) {
            if (!or_sample(g->r_cm[L], c, d, M, &E[L])) E[L] = 0;
            out_hits[(int64_t)p * NL + L] = -1;
        }
        for (i = 0; i < m; i++) {
            int32_t h = hit_idx[q0 + i];
            uint32_t phiM = phi[h] >> (32 - M);
            rel[i] = (int64_t)((phiM - (uint32_t)E[layer[h]]) & mask) - ((int64_t)bp << F);
        }
        for (i = 0; i < m; i++) {
            int64_t c0 = rel[i];
            uint32_t lay_mask = 0;
            int32_t cnt = 0, nl = 0;
            for (j = 0; j < m; j++) {
                if (rel[j] >= c0 && rel[j] < c0 + w) {
                    lay_mask |= 1u << layer[hit_idx[q0 + j]];
                    cnt++;
                }
            }
            for (L = 0; L < NL; L++) nl += (lay_mask >> L) & 1u;
            if (nl > best_l || (nl == best_l && cnt > best_n) || (nl == best_l && cnt == best_n && c0 < best_c)) {
                best_l = nl;
                best_n = cnt;
                best_c = (int32_t)c0;
            }
        }
        out_layers[p] = m > 0 ? best_l : 0;
        for (L = 0; L < NL && m > 0; L++) {
            int32_t pick = -1;
            int64_t pick_d = 0;
            for (j = 0; j < m; j++) {
                int32_t h = hit_idx[q0 + j];
                int64_t dist;
                if (layer[h] != L || !(rel[j] >= best_c && rel[j] < (int64_t)best_c + w)) continue;
                dist = 2 * rel[j] - 2 * (int64_t)best_c - w;
                if (dist < 0) dist = -dist;
                if (pick < 0 || dist < pick_d || (dist == pick_d && h < pick)) {
                    pick = h;
                    pick_d = dist;
                }
            }
            out_hits[(int64_t)p * NL + L] = pick;
            if (pick >= 0) total++;
        }
        free(rel);
    }
    free(phi);
    free(ok);
    return total;
}

/* Threads of the OpenMP loops above (the vote over d0 planes); for timing the oracle at a chosen
 * thread count.  Returns the count in effect. */
int or_set_threads(int n)
{
    if (n > 0) omp_set_num_threads(n);
    return omp_get_max_threads();
}
