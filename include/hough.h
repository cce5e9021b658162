/*
 * hough.h -- C ABI of the MI355X (gfx950) Hough-transform track finder.
 *
 * The method (Halyo et al., "GPU Enhancement of the Trigger to Extend Physics
 * Reach at the LHC"):
 *   Sec. "Proposed Fast Tracking Algorithm", Fig. "hough" caption: every hit
 *     votes for all track parameters it is compatible with; peaks of the
 *     accumulated parameter space are the track candidates (local maxima);
 *   Sec. "Preliminary Results", curved-track paragraph: curved tracks from
 *     the interaction point use a two-parameter space; displaced curved
 *     tracks need a third parameter (here: the transverse impact parameter
 *     d0, so the space is phi0 x q/pT x d0);
 *   Sec. "Preliminary Results", fitting paragraph: the hits of each
 *     candidate are handed to a track fit (here: hough_assign lists them,
 *     hough_fit fits a circle to each list);
 *   Sec. "New Trigger Capabilities": a second transform of the candidates
 *     finds displaced-jet vertices (hough_vertex_*);
 *   Sec. "Preliminary Results", detector paragraph: hits smeared in x and y
 *     (hough_vote_cr: the transform with each hit's own radius);
 *   Sec. "Preliminary Results", data paragraph: hits, parameter space and
 *     peak detection stay resident in GPU memory for the whole event.
 *
 * Discretisation ("fixed-point transform"; the paper is silent on it):
 *   X, Y = round-half-even(x * 2^16), (y * 2^16) as int32 (Q16.16 cm);
 *   Phi  = azimuth of (X, Y) in 32-bit binary angle measure (2^32 = 2 pi) by
 *          30-step integer CORDIC (Volder 1959) with 16 guard bits;
 *   M    = log2(n_phi) + frac_bits;  PhiM = Phi >> (32 - M);
 *   per (layer L, d0 bin l, q/pT bin k), in IEEE double:
 *          q_k = qpt_min + (k + 0.5) * ((qpt_max - qpt_min) / n_qpt)
 *          d_l = d0_min  + (l + 0.5) * ((d0_max  - d0_min)  / n_d0)
 *          c   = -(0.299792458e-2 * B) * q_k,   r = nominal radius of L
 *          A   = (c * (r*r + d*d) + 2.0*d) / (2.0 * r * (1.0 + c*d))
 *          valid iff the denominator > 0 and |A| <= 1
 *          E   = llrint(asin(A) * 2^(M-1) / pi)
 *   vote:  b = ((PhiM - E) mod 2^M) >> frac_bits;  acc[l][k][b] += 1.
 *
 * Conventions
 *   - Every pointer marked (dev) is device memory owned by the caller; the
 *     library never allocates or frees it.  A plan owns only its own
 *     immutable device tables.
 *   - All compute calls are asynchronous on the given stream (NULL = the
 *     default stream), do not synchronise the host, and pass counts between
 *     calls through device memory, so a vote -> peaks -> assign chain can be
 *     captured in a hipGraph.
 *   - Synchronous return codes report argument errors (HOUGH_E_*); data
 *     errors are reported asynchronously in hough_status_t: bad hits are
 *     skipped and counted; an output that exceeds its capacity is truncated
 *     deterministically, its true size is stored and a flag is set.
 *   - A plan may be used concurrently on several streams as long as the
 *     output and workspace buffers of the calls are distinct.
 *   - Results are bit-identical across runs, launch shapes and streams.
 */
#ifndef HOUGH_H
#define HOUGH_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

/* return codes */
#define HOUGH_OK 0
#define HOUGH_E_INVAL (-1)       /* null pointer, negative size, size beyond a limit  */
#define HOUGH_E_UNSUPPORTED (-2) /* grid or geometry outside what the kernels support */
#define HOUGH_E_HIP (-3)         /* a HIP runtime call failed (launch, copy, ...)     */
#define HOUGH_E_NOMEM (-4)       /* plan tables could not be allocated                */
#define HOUGH_E_SMALL_WS (-5)    /* workspace smaller than the size query returned    */

/* status flags */
#define HOUGH_F_PEAK_OVERFLOW 1  /* more peaks than cap: first cap written             */
#define HOUGH_F_PAIR_OVERFLOW 2  /* more hit-candidate pairs than cap: first cap written */
#define HOUGH_F_EVENT_TOO_LARGE 4 /* batch event with more hits than max_hits_per_event:
                                     treated as empty (zero accumulator, no candidates) */

typedef struct {
    int32_t n_layers;          /* 1..32 */
    const double* r_cm;        /* [n_layers] nominal layer radii (host memory, copied) */
    const double* halflen_cm;  /* [n_layers] or NULL (informational)                   */
    double B_tesla;            /* solenoid field along +z                              */
} hough_geometry_t;

typedef struct {
    int32_t n_phi;             /* phi0 bins, power of two, 16..4096                    */
    int32_t n_qpt;             /* q/pT bins (multiple of 64)                           */
    int32_t n_d0;              /* d0 bins (1 = prompt 2-D search)                      */
    int32_t frac_bits;         /* angle bits below one phi0 bin: 7 (16-bit vote counters
                                  in LDS; int32 or int16 accumulator, max_hits_per_event
                                  <= 65535, resp. 32767) or 8 (32-bit counters, int32) */
    double qpt_min, qpt_max;   /* GeV^-1                                               */
    double d0_min, d0_max;     /* cm                                                   */
    int32_t acc_bits;          /* 32 or 16 (int16 requires max_hits_per_event < 32768) */
    int32_t n_cot, n_z0;       /* second-stage r-z grid (0 = none)                     */
    double cot_min, cot_max;   /* cot(theta) range                                     */
    double z0_min, z0_max;     /* cm                                                   */
    int32_t max_hits_per_event;
} hough_grid_t;

/* Structure-of-arrays hits of one event, device memory. */
typedef struct {
    const float* x;            /* (dev) [n] cm */
    const float* y;            /* (dev) [n] cm */
    const float* z;            /* (dev) [n] cm, may be NULL unless hough_zvote is used */
    const uint8_t* layer;      /* (dev) [n] layer id                                   */
    int32_t n;
} hough_hits_t;

typedef struct {
    int32_t l, k, b, votes;    /* d0 bin, q/pT bin, phi0 bin, accumulator value        */
} hough_peak_t;

/* Written by the kernels (device memory, 32 bytes). */
typedef struct {
    int32_t n_hits;            /* hits given to the vote                               */
    int32_t n_bad_hits;        /* skipped: non-finite, |coord| >= 32768 cm, layer out of
                                  range, or at the origin                              */
    int64_t n_votes;           /* hit-votes cast = sum of the accumulator              */
    int32_t n_peaks;           /* true number of candidates (may exceed the capacity)  */
    int32_t flags;             /* HOUGH_F_*                                            */
    int64_t n_pairs;           /* true number of hit-candidate pairs                   */
} hough_status_t;

typedef struct hough_plan hough_plan_t;

/* Launch shapes (results are identical for every valid choice). */
typedef struct {
    int32_t vote_threads;      /* threads per vote workgroup: 256, 512 or 1024            */
    int32_t vote_grid;         /* persistent vote workgroups of a batch (0 = automatic)    */
    int32_t peak_planes;       /* d0 planes walked by one peak-finder thread (1..32);
                                  halved while a launch would give a compute unit
                                  fewer than two workgroups                         */
    int32_t vote_cols;         /* window-table vote: columns per work item, 4..64, a power
                                  of two (0 = automatic)                                 */
    int32_t assign_blocks;     /* assignment workgroups per event (0 = automatic)        */
    int32_t prep_rows;         /* window-table prep: phi0 rows per workgroup, a power of two
                                  16..256 (0 = automatic)                               */
} hough_tuning_t;

/* Create a plan on the current HIP device: validates geometry and grid and
 * builds the per-(layer, d0, q/pT) sample table E (and, with a zvote grid,
 * the arc-length table) in device memory.  Synchronous. */
int hough_plan_create(const hough_geometry_t* geom, const hough_grid_t* grid, hough_plan_t** out);
void hough_plan_destroy(hough_plan_t* plan);

int hough_plan_set_tuning(hough_plan_t* plan, const hough_tuning_t* t);
int hough_plan_get_tuning(const hough_plan_t* plan, hough_tuning_t* t);

/* Kernel timing: while set, every vote kernel launched with this plan (single
 * event or batch) records `start` and `stop` (events created by the caller,
 * timing enabled, may be NULL) with the kernel's own start and end, so their
 * elapsed time is the kernel's duration without launch gaps.  Not for plans
 * used by several threads at once.  NULL, NULL switches it off (default). */
int hough_plan_set_vote_events(hough_plan_t* plan, hipEvent_t start, hipEvent_t stop);
/* The same for the assignment kernel of plans with the window tables (the others ignore it). */
int hough_plan_set_assign_events(hough_plan_t* plan, hipEvent_t start, hipEvent_t stop);

/* Sizes in bytes. */
size_t hough_acc_bytes(const hough_plan_t* plan);             /* n_d0*n_qpt*n_phi*acc_bits/8 */
size_t hough_event_ws_bytes(const hough_plan_t* plan, int32_t max_peaks);
int32_t hough_angle_bits(const hough_plan_t* plan);           /* M */

/* Copy the sample table E[L][l][k] (int32, INT32_MIN = invalid) to host memory
 * `out` of n_layers*n_d0*n_qpt entries.  Synchronous; for tests. */
int hough_plan_table(const hough_plan_t* plan, int32_t* out);

/* a1 -- per-hit preparation: Q16.16 conversion, CORDIC azimuth, validity, and
 * the valid hits sorted by (layer, M-bit angle, hit index) into the workspace.
 * phi_out (dev, may be NULL): [n] 32-bit azimuth of each hit (0 when invalid).
 * ws (dev): at least hough_event_ws_bytes bytes; st (dev): status, reset here. */
int hough_prep(const hough_plan_t* plan, const hough_hits_t* hits, uint32_t* phi_out, void* ws,
               size_t ws_bytes, hough_status_t* st, hipStream_t stream);

/* a1 + a2 -- vote (Sec. "Proposed Fast Tracking Algorithm", Fig. "hough"
 * caption: each hit adds one count to every parameter bin it is compatible
 * with; Sec. "Preliminary Results", curved-track paragraph: the third
 * parameter d0): prep, then acc[l][k][b] (dev, fully overwritten; int32 or
 * int16 per acc_bits, b fastest).  The prepared hits stay in ws for
 * hough_assign.  If n > max_hits_per_event the call returns HOUGH_E_INVAL. */
int hough_vote(const hough_plan_t* plan, const hough_hits_t* hits, void* acc, void* ws, size_t ws_bytes,
               hough_status_t* st, hipStream_t stream);

/* a2 alone -- the vote from hits already prepared in ws by hough_prep (or a
 * previous hough_vote) of the same event; acc as for hough_vote. */
int hough_vote_prepared(const hough_plan_t* plan, void* acc, void* ws, size_t ws_bytes, hough_status_t* st,
                        hipStream_t stream);

/* a3 -- peaks (Fig. "hough" caption: candidate tracks are the local maxima
 * of the accumulated parameter space; the paper gives no neighbourhood, tie
 * rule or threshold, these are readings): bin (l,k,b) is a candidate iff
 * acc >= threshold (>= 1) and,
 * against each of its 3x3x3 neighbours j (phi0 cyclic, q/pT and d0 clipped),
 * acc > acc[j] when j precedes it and acc >= acc[j] otherwise; j precedes
 * when (l_j, k_j) < (l, k) lexicographically or j is bin b-1 (mod n_phi) of
 * the same column.  peaks (dev) [cap] in increasing linear index
 * (l*n_qpt + k)*n_phi + b; st->n_peaks = true count.  Also leaves in ws the
 * number of listed candidates and their CSR offsets for hough_assign
 * (ws of at least hough_event_ws_bytes(plan, cap) bytes). */
int hough_peaks(const hough_plan_t* plan, const void* acc, int32_t threshold, hough_peak_t* peaks,
                int32_t cap, void* ws, size_t ws_bytes, hough_status_t* st, hipStream_t stream);

/* a4 -- assign (Sec. "Preliminary Results", fitting paragraph: the hits of
 * each candidate are handed to a track fit; the paper does not say how hits
 * are associated, this is the reading that a candidate owns exactly the hits
 * that voted for its bin): for each of the first min(listed, cap_peaks) candidates of the
 * preceding hough_peaks call on this ws, the valid hits whose sample at (l, k)
 * falls in bin b (so each list has `votes` entries), ordered layer by layer
 * from the innermost layer, within a layer by the angle inside the bin
 * ((PhiM - E) mod 2^M - b * 2^frac_bits), ties by hit index.
 * CSR: offsets (dev) [cap_peaks+1] (int32; offsets[i] is the prefix sum of the
 * vote counts), hit_idx (dev) [cap_pairs]; entries beyond cap_pairs are not
 * written; st->n_pairs = true total.  Uses the sorted hits left in ws by
 * hough_vote (or hough_prep) of the same event. */
int hough_assign(const hough_plan_t* plan, const hough_peak_t* peaks, int32_t cap_peaks, int32_t* offsets,
                 int32_t* hit_idx, int32_t cap_pairs, void* ws, size_t ws_bytes, hough_status_t* st,
                 hipStream_t stream);

/* a5 -- second-stage r-z vote of every candidate (an extension: the paper's
 * detector model is transverse only, Sec. "Preliminary Results"; this is the
 * straight-line Hough of Sec. "Proposed Fast Tracking Algorithm" applied to
 * the (s, z) plane of each candidate, z = z0 + s cot(theta)).
 * Needs a plan with n_cot, n_z0 > 0.  For candidate p with d0 centre d and
 * curvature c of its (l, k), each hit h of its CSR list with a usable z
 * (finite, |z| < 32768 cm) has Z = rne(z * 2^16) and the arc length to its
 * layer S = llrint(s * 2^16), s = (2/|c|) asin(|c| Lc / 2) (Lc when c = 0),
 * Lc = sqrt(r^2 + d^2 - 2 d r A) the chord from the origin, A as in the
 * sample.  For each cot(theta) row m (Q16.16 centre C_m = llrint(centre *
 * 2^16)) the hit votes into z0 bin j = floor((Z * 2^16 - S * C_m - Z0) / W)
 * when 0 <= j < n_z0, with Z0 = llrint(z0_min * 2^32) and W =
 * llrint(z0 bin width * 2^32) (Q32.32 cm).  out (dev) [cap_peaks][3] gets
 * (m, j, votes) of the fullest bin, lowest m * n_z0 + j on ties;
 * (-1, -1, 0) when no hit votes; (-1, -1, -1) when the candidate's list was
 * cut by cap_pairs.  Candidates: the first min(st->n_peaks, cap_peaks)
 * (st read on the device).  Supported grids: n_z0 <= 512, n_cot * n_z0 <=
 * 65536, W a power of two, the C_m an exact arithmetic progression,
 * |cot| <= 1024, |z0| <= 32768 cm, max_hits_per_event <= 65535 (otherwise
 * hough_plan_create returns HOUGH_E_UNSUPPORTED).  hits->x, y are not read. */
int hough_zvote(const hough_plan_t* plan, const hough_hits_t* hits, const hough_peak_t* peaks, int32_t cap_peaks,
                const int32_t* offsets, const int32_t* hit_idx, int32_t cap_pairs, const hough_status_t* st,
                int32_t* out, hipStream_t stream);

/* Track fit of every listed candidate's hits (Sec. "Preliminary Results",
 * fitting paragraph: the hits of each candidate go on to a fit; the paper
 * names no method).  The fit is the algebraic circle fit of Kasa (IEEE Trans.
 * Instrum. Meas. 25 (1976) 8): the circle x^2 + y^2 + a x + b y + c = 0
 * minimising sum_i (x_i^2 + y_i^2 + a x_i + b y_i + c)^2 over the hits of
 * the candidate's CSR list (hits->x, y in cm, converted to double), the
 * eight moments summed in list order and the 3x3 normal equations solved by
 * Cramer's rule, in IEEE double without contraction (so the result is
 * reproducible bit for bit).  out (dev) [cap_peaks][4] doubles: (xc, yc, R^2,
 * n) = (-a/2, -b/2, xc^2 + yc^2 - c, hits in the list); R^2 = -1 (centre 0)
 * for fewer than 3 hits or a zero determinant; R^2 = -2 when the list was
 * cut by cap_pairs.  Candidates: the first min(st->n_peaks, cap_peaks), st
 * read on the device; offsets / hit_idx as written by hough_assign.
 * Async, stream-ordered; hits->layer and z are not read. */
int hough_fit(const hough_plan_t* plan, const hough_hits_t* hits, const int32_t* offsets, const int32_t* hit_idx,
              int32_t cap_peaks, int32_t cap_pairs, const hough_status_t* st, double* out, hipStream_t stream);

/* Background suppression inside each candidate's bin (Sec. "Preliminary
 * Results", efficiency paragraph: efficiency and purity fall as the number of
 * tracks grows; with many tracks a bin also collects hits of other tracks that
 * cross it).  The track's own hits agree on phi0 far more closely than the bin
 * width, so they sit together in the angle inside the bin.  For each of the
 * first min(st->n_peaks, cap_peaks) candidates, with each listed hit's angle
 * inside the bin rel = ((PhiM - E) mod 2^M) - b * 2^frac_bits (E the sample of
 * its layer at the candidate's (l, k)): among the windows [c, c + window) that
 * begin at a listed hit's rel, the one holding hits of the most distinct
 * layers, then the most hits, then the lowest c; for each layer present in it,
 * the hit nearest the window centre (smallest |2 rel - 2c - window|, ties by
 * the lower hit index).  out_hits (dev) [cap_peaks][n_layers]: that hit or
 * -1; out_layers (dev) [cap_peaks]: layers of the refined list (0 for an empty
 * list, -1 for a list cut by cap_pairs).  Uses the prepared hits left in ws by
 * hough_vote/hough_prep of the same event and the lists of hough_assign;
 * 1 <= window <= 2^frac_bits.  Async, stream-ordered. */
int hough_refine(const hough_plan_t* plan, const hough_peak_t* peaks, int32_t cap_peaks, const int32_t* offsets,
                 const int32_t* hit_idx, int32_t cap_pairs, const void* ws, size_t ws_bytes, const hough_status_t* st,
                 int32_t window, int32_t* out_hits, int32_t* out_layers, hipStream_t stream);

/* The vote with each hit's own radius instead of its layer's (a detector
 * whose hits are smeared off the layer circles, like the paper's model with a
 * 0.4 mm resolution in x and in y, Sec. "Preliminary Results").  Per valid hit
 * (validity and X, Y as for hough_vote): R = floor(sqrt(X^2 + Y^2)) (Q16.16),
 * r = R / 2^16 cm; per (l, k) the sample's A as for the table (IEEE double,
 * same operation order and validity), its arcsine in integers: a =
 * llrint(A * 2^30), b = floor(sqrt(2^60 - a^2)), t = the CORDIC angle of the
 * vector (b, a) as a signed 32-bit binary angle, E = floor((t + 2^(31-M)) /
 * 2^(32-M)); one vote into bin ((PhiM - E) mod 2^M) >> frac_bits.  acc (dev)
 * int32, fully overwritten; st (dev): n_hits, n_bad_hits, n_votes set.  The
 * plan's sample table is not used (the layer only decides validity).
 * Requires acc_bits 32 (HOUGH_E_UNSUPPORTED otherwise).  ALU-bound: every
 * sample is computed, no table.  hough_peaks applies unchanged; the lists
 * come from hough_assign_cr (hough_assign follows the layer table). */
int hough_vote_cr(const hough_plan_t* plan, const hough_hits_t* hits, int32_t* acc, hough_status_t* st,
                  hipStream_t stream);

/* Assignment under the per-hit radius (Sec. "Preliminary Results": the hits
 * of each candidate go on to the fit; here for the transform of
 * hough_vote_cr): for each of the first min(listed, cap_peaks) candidates of
 * the preceding hough_peaks call on `ws` (run on the accumulator that
 * hough_vote_cr wrote for the same hits), the valid hits whose per-hit-radius
 * sample at (l, k) falls in bin b (so each list has `votes` entries), in the
 * order of hough_assign: layer, angle inside the bin, hit index.  CSR output,
 * capacity handling and st->n_pairs as for hough_assign.  ws_cr (dev): a
 * second workspace of hough_assign_cr_ws_bytes(plan, cap_peaks, cap_pairs)
 * bytes (a bin -> candidate map, fill counters and sort keys).  The lists
 * are collected by repeating the vote (same integer arithmetic), so the call
 * costs about as much as hough_vote_cr.  hough_fit applies to its output. */
size_t hough_assign_cr_ws_bytes(const hough_plan_t* plan, int32_t cap_peaks, int32_t cap_pairs);
int hough_assign_cr(const hough_plan_t* plan, const hough_hits_t* hits, const hough_peak_t* peaks, int32_t cap_peaks,
                    int32_t* offsets, int32_t* hit_idx, int32_t cap_pairs, void* ws, size_t ws_bytes, void* ws_cr,
                    size_t ws_cr_bytes, hough_status_t* st, hipStream_t stream);

/* Second Hough transform over the candidates (Sec. "New Trigger Capabilities"
 * and its displaced-jet figures: tracks from one displaced vertex are maxima
 * of the first space lying on one curve, the curve of the vertex; a second
 * transform of the maxima finds it).  Vertex space: n_vr radius rows with
 * centres r_j = r_min + (j + 0.5) * ((r_max - r_min) / n_vr) times n_vphi
 * azimuth bins; bin b_v holds the M-bit angles [b_v, b_v + 1) * 2^(M - log2
 * n_vphi) (M = hough_angle_bits of the first plan).  A first-stage candidate
 * (l, k, b) with votes >= min_votes stands for the helix of its bin centres
 * (d0, q/pT centres; phi0 = M-bit angle b * 2^F + 2^(F-1)); in every row whose
 * sample T = llrint(asin(A(r_j, c, d0)) * 2^(M-1) / pi) is valid (A, validity
 * and operation order as for the first table) it casts one vote for the bin
 * of (phi0 + T) mod 2^M: the azimuth at which the helix, leaving its PCA,
 * meets radius r_j.  acc_v (dev) int32 [n_vr][n_vphi] (azimuth fastest).
 * Vertex peaks: the first stage's peak rule on the grid (1 x n_vr x n_vphi),
 * radius rows clipped, azimuth cyclic; output rows (0, j, b_v, votes). */
typedef struct {
    int32_t n_vr;              /* radius rows: multiple of 64, 64..4096                */
    int32_t n_vphi;            /* azimuth bins: power of two, 16..1024, <= 2^M         */
    double r_min, r_max;       /* cm, 0 <= r_min < r_max <= 32768                      */
    int32_t min_votes;         /* candidates with fewer first-stage votes cast none (>= 1) */
} hough_vertex_grid_t;

typedef struct hough_vertex_plan hough_vertex_plan_t;

/* Builds the table T[l][k][j] (device, n_d0 * n_qpt * n_vr int32) on the
 * current device.  The first plan must outlive the vertex plan.  Synchronous.
 * HOUGH_E_UNSUPPORTED for grids outside the limits above. */
int hough_vertex_plan_create(const hough_plan_t* plan, const hough_vertex_grid_t* vgrid, hough_vertex_plan_t** out);
void hough_vertex_plan_destroy(hough_vertex_plan_t* vplan);
/* Candidate ranges counted apart and then added (launch shape only: results
 * are identical for every value; raised to ceil(cap_peaks / 65535) when
 * smaller).  Default: enough workgroups for every compute unit. */
int hough_vertex_set_groups(hough_vertex_plan_t* vplan, int32_t groups);
int32_t hough_vertex_get_groups(const hough_vertex_plan_t* vplan);
/* Workspace of hough_vertex_vote for a candidate capacity, and of
 * hough_vertex_peaks for a vertex-candidate capacity (two separate buffers
 * or one reused in stream order). */
size_t hough_vertex_vote_ws_bytes(const hough_vertex_plan_t* vplan, int32_t cap_peaks);
size_t hough_vertex_peaks_ws_bytes(const hough_vertex_plan_t* vplan, int32_t cap_vpeaks);
/* Vote the first min(st->n_peaks, cap_peaks) candidates of `peaks` (dev, as
 * written by hough_peaks on the first plan; st read on the device) into acc_v
 * (dev, fully overwritten).  Candidates whose (l, k, b) lies outside the first
 * grid cast nothing.  st_v (dev) is reset: n_hits = candidates given, n_votes
 * = votes cast = sum of acc_v, other fields 0.  Async, stream-ordered. */
int hough_vertex_vote(const hough_vertex_plan_t* vplan, const hough_peak_t* peaks, int32_t cap_peaks,
                      const hough_status_t* st, int32_t* acc_v, void* ws, size_t ws_bytes, hough_status_t* st_v,
                      hipStream_t stream);
/* Local maxima of acc_v with acc_v >= threshold (>= 1): vpeaks (dev) [cap] in
 * increasing j * n_vphi + b_v; st_v->n_peaks = true count, flags as for
 * hough_peaks.  ws of hough_vertex_peaks_ws_bytes(vplan, cap) bytes. */
int hough_vertex_peaks(const hough_vertex_plan_t* vplan, const int32_t* acc_v, int32_t threshold,
                       hough_peak_t* vpeaks, int32_t cap, void* ws, size_t ws_bytes, hough_status_t* st_v,
                       hipStream_t stream);
/* The same for n_events events at once (1..65535): candidate lists at peaks +
 * e * cap_peaks with statuses st[e] (as hough_run_batch writes them), vertex
 * spaces at acc_v + e * n_vr * n_vphi, statuses st_v[e]; vertex candidates at
 * vpeaks + e * cap.  Results equal the single-event calls per event. */
size_t hough_vertex_batch_vote_ws_bytes(const hough_vertex_plan_t* vplan, int32_t n_events, int32_t cap_peaks);
size_t hough_vertex_batch_peaks_ws_bytes(const hough_vertex_plan_t* vplan, int32_t n_events, int32_t cap_vpeaks);
int hough_vertex_vote_batch(const hough_vertex_plan_t* vplan, int32_t n_events, const hough_peak_t* peaks,
                            int32_t cap_peaks, const hough_status_t* st, int32_t* acc_v, void* ws, size_t ws_bytes,
                            hough_status_t* st_v, hipStream_t stream);
int hough_vertex_peaks_batch(const hough_vertex_plan_t* vplan, int32_t n_events, const int32_t* acc_v,
                             int32_t threshold, hough_peak_t* vpeaks, int32_t cap, void* ws, size_t ws_bytes,
                             hough_status_t* st_v, hipStream_t stream);
/* Copy T to host memory `out` (n_d0 * n_qpt * n_vr entries).  Synchronous; for tests. */
int hough_vertex_table(const hough_vertex_plan_t* vplan, int32_t* out);

/* Copy the arc-length table S[L][l][k] (int32 Q16.16, -1 = invalid) of a
 * plan with an r-z grid to host memory `out` (n_layers*n_d0*n_qpt entries).
 * Synchronous; for tests. */
int hough_plan_arclen_table(const hough_plan_t* plan, int32_t* out);

/* a7 -- batched form: many events of uneven size in one launch chain.  The
 * hits of all events are packed (CSR: event e owns hits [hit_offsets[e],
 * hit_offsets[e+1])); every per-event output is strided by its capacity.
 * The vote is one persistent kernel that pulls (event, slab of 64 columns)
 * items from a device work queue, largest events first (Sec. "Preliminary
 * Results", data paragraph: each GPU processes one event after another; here
 * the events of a batch share the GPU).  With `zvote` set (plan with an r-z
 * grid, z given) the chain ends with hough_zvote of every event.  Results of
 * each event are identical to the single-event calls.  Stream-ordered; capturable in a hipGraph. */
typedef struct {
    const float* x;            /* (dev) packed hits of all events                        */
    const float* y;
    const float* z;            /* may be NULL                                            */
    const uint8_t* layer;
    const int32_t* hit_offsets;/* (dev) [n_events + 1]                                   */
    int32_t n_events;
    int32_t threshold;         /* peak threshold (>= 1)                                  */
    int32_t cap_peaks;         /* per event                                              */
    int32_t cap_pairs;         /* per event                                              */
    void* acc;                 /* (dev) n_events x hough_acc_bytes                       */
    hough_peak_t* peaks;       /* (dev) n_events x cap_peaks                             */
    int32_t* offsets;          /* (dev) n_events x (cap_peaks + 1)                       */
    int32_t* hit_idx;          /* (dev) n_events x cap_pairs                             */
    void* ws;                  /* (dev) hough_batch_ws_bytes(plan, n_events, cap_peaks)  */
    size_t ws_bytes;
    hough_status_t* status;    /* (dev) n_events                                         */
    int32_t* zvote;            /* (dev) n_events x cap_peaks x 3, or NULL: no r-z stage  */
} hough_batch_t;

size_t hough_batch_ws_bytes(const hough_plan_t* plan, int32_t n_events, int32_t cap_peaks);
int hough_run_batch(const hough_plan_t* plan, const hough_batch_t* batch, hipStream_t stream);

/* hough_run_batch for callers that cannot allocate device memory (code under
 * hipGraph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the workspace is a scratch array the library holds in device memory, one
 * copy of HOUGH_NOALLOC_SCRATCH_BYTES per GPU, kept until the process ends
 * (its address is looked up when a plan is created on that GPU).  The call
 * allocates nothing.  batch->ws must be NULL and ws_bytes 0 (HOUGH_E_INVAL
 * otherwise); hough_batch_ws_bytes(plan, n_events, cap_peaks) must not
 * exceed HOUGH_NOALLOC_SCRATCH_BYTES (HOUGH_E_SMALL_WS otherwise; e.g. a few
 * 512x256x64 events or one 1024x512x128 event).  HOUGH_E_HIP if the scratch
 * array of the plan's GPU could not be located.  Every call on one GPU uses
 * the same array, which keeps the last call's contents (the chain clears
 * what it needs zeroed itself): calls that overlap in time on one GPU (on
 * different streams or from different host threads) race and must be
 * serialised by the caller.  Results equal hough_run_batch's. */
#define HOUGH_NOALLOC_SCRATCH_BYTES (64 << 20)
int hough_run_batch_noalloc(const hough_plan_t* plan, const hough_batch_t* batch, hipStream_t stream);

/* Track fit (as hough_fit) of every listed candidate of every event of a
 * batch after hough_run_batch: hits, offsets, hit lists and statuses taken
 * from `batch`; out (dev) [n_events][cap_peaks][4] doubles.  Results equal
 * hough_fit on each event alone. */
int hough_fit_batch(const hough_plan_t* plan, const hough_batch_t* batch, double* out, hipStream_t stream);

/* The batched chain captured once into a hipGraph and replayed: buffers are
 * bound at capture time (refill the same buffers with new events between
 * launches).  `stream` must not be the NULL stream. */
typedef struct hough_graph hough_graph_t;
int hough_batch_graph_create(const hough_plan_t* plan, const hough_batch_t* batch, hipStream_t stream,
                             hough_graph_t** out);
int hough_graph_launch(hough_graph_t* graph, hipStream_t stream);
void hough_graph_destroy(hough_graph_t* graph);

const char* hough_strerror(int code);

#ifdef __cplusplus
}
#endif
#endif /* HOUGH_H */
