/*
 * tpcf.h -- C ABI of libtpcf.so: the anisotropic three-point correlation
 * function (3PCF) estimator of arXiv:2408.03036, Sec. 4.2, on one MI355X.
 *
 * The library computes, for a periodic box of side L with points x_i and
 * weights w_i (1 for data; -N_D/N_R for randoms in the data-minus-randoms
 * field of the Szapudi-Szalay estimator, eq. (ssest)):
 *
 *   a_lm(p, b)  = sum over neighbours j of p with |x_j - x_p| in radial bin b
 *                 of w_j conj(Y_lm(rhat_pj))                            eq. (alm)
 *   NNN^m_{l1 l2}(b1, b2) = sum_p w_p [a_{l1 m}(p,b1) conj(a_{l2 m}(p,b2))
 *                 - delta_{b1 b2} sum_j w_j^2 conj(Y_{l1 m}) Y_{l2 m}]
 *                 (m = m' because the line of sight is the fixed z axis;
 *                  eq. (measured_mult) averaged over positions x)
 *   zeta_{l1 l2 L}(b1, b2) = 4 pi sqrt((2l1+1)(2l2+1)) (2L+1) H_{l1 l2 L}
 *                 sum_m (l1 l2 L; m -m 0) (-1)^m NNN^m / RRR(b1, b2)
 *                 (eq. (slep2sugy), normalised as the coefficient of the
 *                  tripolar basis of eq. (TSHbasis)), with the analytic
 *                 periodic-box random-triplet count
 *                 RRR = N_D (N_D-1)(N_D-2) V_b1 V_b2 / L^6.
 * Y_lm is orthonormal; bins are half-open [e_b, e_{b+1}); the minimum-image
 * separation is used; pairs at zero separation and degenerate triangles
 * (j == k) are excluded.
 *
 * The same handle also measures the anisotropic two-point function of Sec.
 * 4.1 on the neighbour grid of step 1 (tpcf_xi_count, tpcf_xi_multipoles):
 *
 *   DD(b, k)  = ordered pairs (p, j != p) with |x_j - x_p| in radial bin b and
 *               mu = (z_j - z_p) / |x_j - x_p| (line of sight z) in bin k of
 *               nmu equal bins over [-1, 1]
 *   xi(r_b, mu_k) = DD(b, k) / RR(b, k) - 1,  RR(b, k) = N (N-1) V_b / (nmu L^3)
 *               (the natural estimator of eq. (xi_natest) with the analytic
 *                random pairs of a periodic box)
 *   xi_l(r_b) = (2l+1)/2 sum_k xi(r_b, mu_k) * integral of P_l over bin k
 *               (eq. (xi_meas_leg) with xi constant inside a mu bin).
 *
 * Conventions for every call:
 *  - Pointers prefixed d_ are DEVICE pointers on the handle's device (for
 *    example torch.Tensor.data_ptr()); h_ are HOST pointers. The caller owns
 *    every buffer it passes; the library owns its workspace.
 *  - Work is enqueued on the HIP stream given to tpcf_create; device outputs
 *    are valid once that stream has reached them (tpcf_sync waits for it).
 *  - Every call returns a tpcf_status; no C++ exception crosses the ABI.
 *    Arguments are validated before any device work is enqueued.
 *    tpcf_last_error() gives a message for the last failing call.
 *  - A handle is used by one host thread at a time.
 *  - Lengths are in the units of `box` (Mpc/h in the paper).
 */
#ifndef TPCF_H
#define TPCF_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct tpcf_handle_s* tpcf_handle;

typedef enum {
    TPCF_OK = 0,
    TPCF_ERR_ARG = -1,     /* invalid argument (NULL pointer, bad size, bad triple) */
    TPCF_ERR_RANGE = -2,   /* configuration outside the supported range              */
    TPCF_ERR_ALLOC = -3,   /* device memory could not be obtained or over budget     */
    TPCF_ERR_DEVICE = -4,  /* a HIP call failed, or non-finite input positions       */
    TPCF_ERR_STATE = -5    /* call out of order (e.g. contract before accumulate)    */
} tpcf_status;

/* Arithmetic of the pair pass and of the contraction. */
typedef enum {
    TPCF_PREC_FP64 = 0,         /* FP64 pair pass, FP64 MFMA contraction                      */
    TPCF_PREC_FP32 = 1,         /* FP32 pair pass, FP32 MFMA contraction, FP64 final sums     */
    TPCF_PREC_MIXED_BF16X3 = 2, /* FP32 pair pass, split-BF16 contraction: x = hi + lo (BF16),
                                   products hi.hi + hi.lo + lo.hi on BF16 MFMA, FP32
                                   accumulation per subchunk, FP64 final sums. With weights
                                   (d_w given) the six-product split of MIXED_BF16X6 is
                                   used: data and random terms cancel in the sum over
                                   primaries and would magnify the three-product error   */
    TPCF_PREC_MIXED_BF16X6 = 3  /* as above with x = hi + mid + lo and six products (every
                                   product above 2^-24 relative): FP32-level accuracy for
                                   sparse bins at twice the BF16 MFMA work                    */
} tpcf_precision;

enum {
    TPCF_F_KEEP_DEGENERATE = 1u, /* keep j == k terms (default: distinct triplets only)     */
    TPCF_F_PAPER_LITERAL = 2u,   /* output eq. (slep2sugy) exactly as printed, applied to the
                                    orthonormal-Y coefficients (4 pi)^2 NNN^m / RRR; equals the
                                    default output times 4 pi / sqrt((2l1+1)(2l2+1))          */
    TPCF_F_ISOTROPIC = 4u        /* isotropic schedule (the L = 0 case of eq. (TripoSH), Sec.
                                    2.3): the contraction forms only the l1 = l2 blocks of NNN^m,
                                    in FP64 (MFMA) from the pair pass of the chosen precision,
                                    and tpcf_multipoles / tpcf_run_catalogs accept only (l, l, 0)
                                    triples. By the addition theorem zeta_{l l 0}(r1, r2) is then
                                    the Legendre coefficient zeta_l of zeta(r1, r2, cos theta_12).
                                    Exported NNN^m is zero off the l1 = l2 blocks. nbins <= 32. */
};

typedef struct {
    double box;              /* L > 0, finite; the box is periodic in x, y and z             */
    int32_t nbins;           /* 1 .. 32 radial bins (a bin's per-primary counters and
                                predicted regions are one 32-entry LDS row per primary in
                                the binning kernel)                                           */
    const double* h_edges;   /* nbins+1 strictly increasing edges, edges[0] >= 0,
                                edges[nbins] <= box/2 (minimum image); copied at create       */
    int32_t lmax;            /* 0 .. 16. The harmonic pass keeps the a_lm of a (primary,
                                bin) list in one lane's registers; above lmax 10 (FP32) or
                                6 (FP64) it splits the m range over 2 launches, and from 13
                                over 3 (FP32) or 4 (FP64), each rereading the lists. With
                                weights and nbins (lmax + 1) > 512 the split-BF16
                                precisions contract on FP32 MFMA.                          */
    int32_t precision;       /* tpcf_precision                                                */
    uint32_t flags;          /* TPCF_F_* bits                                                 */
    int32_t grid_refine;     /* cells per r_max along an axis for the neighbour grid,
                                1 .. 4; 0 = automatic                                         */
    int64_t workspace_limit; /* device bytes the handle may hold; 0 = 64 GiB                  */
} tpcf_config;

/* Creates a handle bound to `device` (HIP ordinal) and `hip_stream`
 * (a hipStream_t, or NULL for the null stream). Copies *cfg. */
tpcf_status tpcf_create(const tpcf_config* cfg, int device, void* hip_stream, tpcf_handle* out);

/* Releases the handle and its device workspace (waits for its stream). NULL is a no-op. */
void tpcf_destroy(tpcf_handle h);

/* Message of the last failing call on h (static string for h == NULL); never NULL. */
const char* tpcf_last_error(tpcf_handle h);

/*
 * Step 1 -- neighbour grid (the linked-list partition of Sec. 4.1, built as a
 * counting sort of the points by cell).
 *  d_pos : n x 3 float64, row-major; positions are wrapped into [0, box).
 *  d_w   : n float64 weights, or NULL for all ones.
 *  n     : number of points (every point is also a primary), 1 .. 2^27.
 *  n_data: N_D used in RRR (the number of data points), >= 3.
 * The buffers must stay valid until tpcf_alm_accumulate has been enqueued.
 * Non-finite positions make the next call return TPCF_ERR_DEVICE.
 */
tpcf_status tpcf_build_grid(tpcf_handle h, const double* d_pos, const double* d_w,
                            int64_t n, int64_t n_data);

/*
 * Step 2 -- pair pass: for every primary, every neighbour in the shells;
 * accumulates a_lm(p, b) (eq. (alm)) and the degenerate-triangle moments
 * sum_j w_j^2 P_L(cos theta_pj), L <= 2 lmax. Requires tpcf_build_grid.
 * The chunks of primaries run without host round trips; the call waits for
 * the stream once, after the last chunk, to learn whether the hit lists ran
 * out of room (strong clustering), and then runs the pass again with twice
 * the room (which the handle keeps for later calls). TPCF_ERR_ALLOC when the
 * room cannot grow within the workspace limit or 16e9 entries.
 */
tpcf_status tpcf_alm_accumulate(tpcf_handle h);

/*
 * Copies a_lm(p, b) = sum_j w_j conj(Y_lm(rhat_pj)) of primaries
 * [first, first+count) (indices into the d_pos passed to tpcf_build_grid)
 * to d_out: count x nbins x (lmax+1) x (lmax+1) complex (re, im) float64,
 * entry [p][b][l][m] for 0 <= m <= l (other entries zero). Requires step 2.
 */
tpcf_status tpcf_get_alm(tpcf_handle h, int64_t first, int64_t count, double* d_out);

/*
 * Step 3 -- contraction: NNN^m_{l1 l2}(b1, b2) summed over all primaries,
 * real part (the imaginary part does not enter any even-parity multipole),
 * degenerate triangles removed unless TPCF_F_KEEP_DEGENERATE.
 * d_nnn_out: NULL, or (lmax+1)^3 x nbins x nbins float64 laid out
 * [m][l1][l2][b1][b2] (entries with l1 < m or l2 < m are zero); refused
 * with TPCF_ERR_STATE after a tpcf_run_catalogs that stopped the self
 * moments, skipped blocks, or whose last group held several catalogues (the
 * step calls give every catalogue's).
 * Requires step 2.
 */
tpcf_status tpcf_contract(tpcf_handle h, double* d_nnn_out);

/*
 * Step 4 -- multipoles zeta_{l1 l2 L}(b1, b2) for n_mult triples.
 *  h_l1l2L: host array n_mult x 3 of (l1, l2, L) with l1, l2 <= lmax,
 *           |l1 - l2| <= L <= l1 + l2 and l1 + l2 + L even (eq. (TripoSH)).
 *  d_out  : n_mult x nbins x nbins float64.
 * Requires step 3, and a handle whose sums are those of one catalogue: after
 * a tpcf_run_catalogs whose last group held several, TPCF_ERR_STATE (that
 * call returns their multipoles).
 */
tpcf_status tpcf_multipoles(tpcf_handle h, int32_t n_mult, const int32_t* h_l1l2L,
                            double* d_out);

/*
 * Steps 1-4 for ncat catalogues in one batched pass (the mock-catalogue use of
 * Sec. 4.2 and 4.3). Catalogue c holds h_n[c] points stored after those of
 * catalogues 0..c-1 in d_pos (sum h_n rows x 3 float64) and d_w (NULL = ones),
 * and uses h_n_data[c] in its RRR. Results go to d_out, ncat x n_mult x nbins
 * x nbins float64. Catalogues are processed in groups that fit the workspace
 * limit; results do not depend on the grouping.
 * When every requested L is <= lmax, the self moments of order above lmax are
 * not accumulated (they cancel from such multipoles, the 3j symbols of a
 * multipole being orthogonal over m); the results equal those of steps 1-4 bit
 * for bit. Until the next tpcf_build_grid the handle then refuses, with
 * TPCF_ERR_STATE, a tpcf_contract export of NNN^m and tpcf_multipoles triples
 * with L > lmax. Likewise the split-BF16 contraction of such a run forms only
 * the (l1, l2) blocks that its multipoles couple (|l1 - l2| up to the largest
 * among them, each multipole needing |l1 - l2| <= L): until the next
 * tpcf_build_grid, triples with a larger |l1 - l2| and the per-m export are
 * refused with TPCF_ERR_STATE.
 * A catalogue with a non-finite coordinate does not stop the others: its
 * results are NaN, its status (tpcf_catalog_status) TPCF_ERR_DEVICE, the other
 * catalogues' results are complete and equal those of a batch without it, and
 * the call returns TPCF_ERR_DEVICE naming the catalogues. Any other error
 * leaves d_out undefined.
 */
tpcf_status tpcf_run_catalogs(tpcf_handle h, int32_t ncat, const int64_t* h_n,
                              const int64_t* h_n_data, const double* d_pos, const double* d_w,
                              int32_t n_mult, const int32_t* h_l1l2L, double* d_out);

/*
 * Status of each catalogue of the last tpcf_run_catalogs that returned after
 * its argument checks: h_status (host, ncat int32) gets TPCF_OK or
 * TPCF_ERR_DEVICE (non-finite positions). ncat must equal that call's.
 * TPCF_ERR_ARG on a NULL h_status or a different ncat.
 */
tpcf_status tpcf_catalog_status(tpcf_handle h, int32_t ncat, int32_t* h_status);

/*
 * Anisotropic 2PCF pair counts DD(r, mu) (Sec. 4.1) of the catalogue given to
 * tpcf_build_grid, which must have been built without weights (d_w = NULL);
 * the radial bins are the handle's edges. Requires tpcf_build_grid.
 *  nmu     : mu bins over [-1, 1], 1 .. 4096, with nbins * nmu <= 16384.
 *            With r^2 = dx*dx + dy*dy + dz*dz and mu = dz / sqrt(r^2), the
 *            bin is floor((mu + 1) nmu / 2) evaluated in double, clamped to
 *            nmu - 1 (mu = 1 falls in the last bin).
 *  d_counts: nbins x nmu int64 (device), [b][k], overwritten. Every ordered
 *            pair is counted, so DD(b, k) and DD(b, nmu-1-k) differ only
 *            through pairs on a mu edge.
 * Exact: the counts equal those of a double-precision evaluation of every pair.
 */
tpcf_status tpcf_xi_count(tpcf_handle h, int32_t nmu, int64_t* d_counts);

/*
 * Legendre multipoles xi_l(r_b) (eq. (xi_meas_leg)) of the natural estimator
 * from pair counts d_counts (nbins x nmu int64, device, as written by
 * tpcf_xi_count) of a catalogue of n_data >= 2 points in the handle's box.
 *  h_ells: host array of n_ell (1 .. 64) orders l in 0 .. 60.
 *  d_out : n_ell x nbins float64 (device).
 * Needs no earlier step; reads d_counts on the handle's stream.
 */
tpcf_status tpcf_xi_multipoles(tpcf_handle h, int32_t nmu, const int64_t* d_counts, int64_t n_data,
                               int32_t n_ell, const int32_t* h_ells, double* d_out);

/*
 * Autotuner of the neighbour grid. Times, on the sample catalogue (d_pos,
 * d_w, n, n_data as for tpcf_build_grid), the pair pass (steps 1-2, nmu = 0)
 * or the 2PCF pair counts (nmu > 0, unit weights) for every admissible grid
 * refinement 1 .. 4 (cells of r_max / k), and keeps the fastest on the handle
 * for later grids (it replaces the config's grid_refine). Results do not
 * depend on the refinement: bin decisions are exact at every one.
 *  h_refine: the refinement chosen.  h_ms: NULL, or 4 entries: the time of
 *  each refinement in ms (-1 where it is not admissible for the box).
 * The sample's grid is not kept: call tpcf_build_grid afterwards.
 */
tpcf_status tpcf_autotune(tpcf_handle h, const double* d_pos, const double* d_w, int64_t n, int64_t n_data,
                          int32_t nmu, int32_t* h_refine, double* h_ms);

/*
 * Launch plan of the estimator, chosen by tpcf_autotune_plan or set by the
 * caller (for example from a cache of plans keyed by device, precision, lmax,
 * bins and catalogue density). Results do not depend on the refinement (every
 * bin decision is exact); the list mode and the contraction step change only
 * the order of FP32 sums.
 *  grid_refine:   cells per r_max along an axis, 1 .. 4; 0 = automatic.
 *  list_mode:     harmonic pass: 0 one lane per (primary, bin) list, 1 one
 *                 wavefront per list (FP32 paths with lmax <= 6; elsewhere
 *                 the lane kernel runs), -1 = by the predicted list length.
 *  contract_step: longest step (primaries) of the split-BF16 contraction:
 *                 16, 32, 64 or 128, or 0 = up to 512. Each m takes the
 *                 longest step up to this that its columns' staging fits
 *                 (the narrow high-m operands take the longest). Other
 *                 precisions ignore it.
 *  ms:            (tpcf_autotune_plan) the timed pair pass and contraction of
 *                 the sample with this plan, in ms.
 */
typedef struct {
    int32_t grid_refine;
    int32_t list_mode;
    int32_t contract_step;
    int32_t reserved;
    double ms;
} tpcf_plan;

/*
 * Times steps 1-3 (grid build, pair pass, contraction) of a sample batch
 * (ncat, h_n, h_n_data, d_pos, d_w as for tpcf_run_catalogs; for example the
 * batch itself, or one representative catalogue) with every admissible grid
 * refinement, both list modes where the wavefront kernel exists, and for the
 * non-isotropic split-BF16 precisions the longest contraction step and 64;
 * keeps the fastest plan on the handle and returns it.
 *  h_ms: NULL, or 16 entries receiving the time (ms) of each candidate at
 *        [((grid_refine - 1) * 2 + list_mode) * 2 + (contract_step ? 1 : 0)],
 *        -1 where it was not run (or its lists did not fit the workspace).
 * The sample's grid and sums are not kept: build or run afterwards.
 */
tpcf_status tpcf_autotune_plan(tpcf_handle h, int32_t ncat, const int64_t* h_n, const int64_t* h_n_data,
                               const double* d_pos, const double* d_w, tpcf_plan* h_plan, double* h_ms);
/* Applies a plan (out-of-range fields give TPCF_ERR_RANGE); it takes effect
 * from the next tpcf_build_grid or tpcf_run_catalogs. */
tpcf_status tpcf_set_plan(tpcf_handle h, const tpcf_plan* h_plan);
/* The handle's current plan (ms = 0). */
tpcf_status tpcf_get_plan(tpcf_handle h, tpcf_plan* h_plan);

/*
 * Szapudi-Szalay estimator with explicit randoms (eq. (ssest)), isotropic
 * multipoles: edge correction by the random triplet counts. With N_l the
 * multipoles (l, l, 0) of a data-minus-randoms run (weights 1 and -N_D/N_R,
 * n_data = N_D) and R_l those of a run on the randoms alone (n_data = N_R),
 * both on the handle's bins, the relation N(cos t) = zeta(cos t) R(cos t)
 * between the triplet counts as functions of the opening angle gives
 *   N_l = sum_{l'} M_{l l'} zeta_{l'},  M_{l l'} = sum_{l''} (2l+1) (l l' l''; 0 0 0)^2 R_{l''}
 * (the relation of Slepian & Eisenstein 2015; R truncated at n_ell - 1),
 * solved for zeta at every (b1, b2) in FP64.
 *  d_N, d_R, d_out: device, n_ell x nbins x nbins float64 ([l][b1][b2], l = 0 .. n_ell-1,
 *                   as tpcf_multipoles writes the triples (l, l, 0) in order).
 *  n_ell in 1 .. 25. A singular coupling matrix gives TPCF_ERR_RANGE.
 *  Synchronises the stream.
 */
tpcf_status tpcf_edge_correct_isotropic(tpcf_handle h, int32_t n_ell, const double* d_N, const double* d_R,
                                        double* d_out);

/*
 * Szapudi-Szalay estimator with explicit randoms (eq. (ssest)), anisotropic
 * multipoles: edge correction of the tripolar multipoles by the random triplet
 * counts. Let N and R be the triplet counts of a data-minus-randoms run
 * (weights 1 and -N_D/N_R) and of a run on the randoms alone, each a function of
 * the two sides' directions (r1, r2) in a bin pair (b1, b2), with coefficients
 * N^m_{l1 l2} and R^m_{l1 l2} in the orthonormal basis Y_l1m(r1) conj(Y_l2m(r2))
 * (the exported NNN^m of tpcf_contract, each divided by its analytic RRR). The
 * estimator N = zeta R, taken at every pair of directions, gives
 *   N^m_{l1 l2} = sum zeta^{m'}_{l1' l2'} R^{m-m'}_{l1'' l2''} g(l1 m; l1' m'; l1'') g(l2 m; l2' m'; l2''),
 *   g(l m; l' m'; l'') = integral of conj(Y_lm) Y_l'm' Y_l'',m-m' over the sphere,
 * with every l truncated at the handle's lmax; it is solved for zeta at every
 * (b1, b2) in FP64 (Gaussian elimination with partial pivoting). Only real
 * coefficients enter (the export holds the real parts): the reflection-
 * symmetric sector, whose coefficients satisfy X^{-m} = X^m.
 *  d_nnn_N, d_nnn_R: device, (lmax+1)^3 x nbins x nbins float64 each, the
 *            exports of tpcf_contract of the two runs, made on handles with
 *            this handle's box, bins and lmax (not checked).
 *  n_data_N, n_data_R: N_D of the data-minus-randoms run and N_R of the randoms
 *            run (their RRR normalisations), >= 3.
 *  h_l1l2L, n_mult, d_out: multipoles of zeta as for tpcf_multipoles
 *            (n_mult x nbins x nbins), or d_out = NULL for none.
 *  d_zeta:   NULL, or device (lmax+1)^3 x nbins x nbins float64 receiving the
 *            corrected coefficients zeta^m in the export layout.
 *  lmax <= 10 (TPCF_ERR_RANGE otherwise). A singular system gives
 *  TPCF_ERR_RANGE. Synchronises the stream.
 */
tpcf_status tpcf_edge_correct(tpcf_handle h, const double* d_nnn_N, int64_t n_data_N, const double* d_nnn_R,
                              int64_t n_data_R, int32_t n_mult, const int32_t* h_l1l2L, double* d_out,
                              double* d_zeta);

/*
 * Covariance step of Sec. 4.3, for measurements of a suite of mock catalogues.
 *
 * tpcf_triangle_index: host helper building a 3PCF data vector. For each
 * multipole row t of h_rows (indices into an n_mult x nbins x nbins output
 * block such as one catalogue of tpcf_run_catalogs) it lists the triangle
 * configurations in the order of the flattened (r1, r2) grid: unique
 * configurations r1 < r2 (bin centres), side difference r2 - r1 >= eta * dr and
 * shortest side r1 >= r_min (Sec. 4.3 and 5). Bins must be of equal width dr.
 *  h_offsets: capacity entries (t nbins + b1) nbins + b2; h_count: number of
 *  configurations (also when capacity is 0, then h_offsets may be NULL).
 *  Returns TPCF_ERR_RANGE when capacity (> 0) is too small or the bins are not
 *  of equal width. Needs no handle and no device.
 */
tpcf_status tpcf_triangle_index(int32_t nbins, const double* h_edges, double eta, double r_min, int32_t n_rows,
                                const int32_t* h_rows, int64_t capacity, int64_t* h_offsets, int64_t* h_count);

/*
 * Mean and unbiased covariance of n_mocks data vectors (eq. (covariance)):
 *   C_ij = 1/(N_m - 1) sum_k (d_i^k - dbar_i)(d_j^k - dbar_j).
 *  d_src    : device, n_mocks rows of `stride` float64 (for example the output
 *             of tpcf_run_catalogs, stride = n_mult nbins nbins).
 *  h_offsets: host, n_d offsets into a row giving the data vector (NULL: the
 *             first n_d entries); each in 0 .. stride-1.
 *  d_mean   : device, n_d float64, or NULL.  d_cov: device, n_d x n_d float64.
 * FP64 throughout (the products on FP64 MFMA); the mean is summed in mock order.
 */
tpcf_status tpcf_covariance(tpcf_handle h, int32_t n_mocks, int64_t stride, const double* d_src, int32_t n_d,
                            const int64_t* h_offsets, double* d_mean, double* d_cov);

/*
 * tpcf_covariance without any device allocation, for callers that cannot
 * allocate (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc). Same kernels and same results, bit for bit, as
 * tpcf_covariance on the same inputs; it calls no hipMalloc or hipFree.
 *  d_offsets: DEVICE array of n_d int64 offsets into a row, or NULL (the first
 *             n_d entries). The host cannot check device offsets: an offset
 *             outside 0 .. stride-1 reads nothing and gives NaN in its row and
 *             column of d_cov (and in d_mean).
 *  Other arguments as for tpcf_covariance.
 * The gathered data vectors and the partial products live in a static device
 * array of 32 MiB (32 << 20 bytes) that every device the library runs on holds
 * until the process ends: 8 (n_mocks n_d + P) bytes must fit it, P being the
 * partial products (n_mocks = 3000, n_d = 336 needs 24.3 MB). Larger inputs are
 * refused with TPCF_ERR_RANGE before any device work. Every call on one device
 * uses that device's one array: calls that overlap on one device (on two
 * streams, or from two handles) race and give wrong results; calls in one
 * stream's order do not. Nothing in the array needs to start at zero.
 */
tpcf_status tpcf_covariance_noalloc(tpcf_handle h, int32_t n_mocks, int64_t stride, const double* d_src, int32_t n_d,
                                    const int64_t* d_offsets, double* d_mean, double* d_cov);

/*
 * Precision matrix with the Hartlap correction (eq. (Hartlap)):
 *   d_prec = (N_m - N_d - 2)/(N_m - 1) * inverse(d_cov),
 * by a Gauss-Jordan sweep in FP64 (d_prec may equal d_cov: in place).
 * n_d in 1 .. 4096 and n_mocks >= n_d + 3 (else TPCF_ERR_RANGE); a matrix that
 * is not positive definite gives TPCF_ERR_RANGE. Synchronises the stream.
 */
tpcf_status tpcf_precision_matrix(tpcf_handle h, int32_t n_d, const double* d_cov, int32_t n_mocks, double* d_prec);

/*
 * Percival correction of the parameter variances (eqs. (Perc1), (Perc)):
 *   m1 = (1 + B (N_d - N_p)) / (1 + A + B (N_p + 1)),
 *   A = 2 / ((N_m - N_d - 1)(N_m - N_d - 4)),  B = (N_m - N_d - 2) / ((N_m - N_d - 1)(N_m - N_d - 4)).
 * Requires n_mocks >= n_d + 5. Host only.
 */
tpcf_status tpcf_percival_m1(int32_t n_mocks, int32_t n_d, int32_t n_params, double* h_m1);

/* Waits for all work enqueued by h. */
tpcf_status tpcf_sync(tpcf_handle h);

/* Ordered in-shell pairs counted by the last pair pass (valid after tpcf_sync). */
tpcf_status tpcf_pair_count(tpcf_handle h, int64_t* h_out);

/*
 * Primaries whose neighbours were binned a second time with exact counts since
 * the handle was created. The binning pass gives each (primary, bin) a region
 * sized from the local density its cell's stencil shows; a primary with more
 * neighbours in some bin than its region holds (strong clustering) is redone
 * with exact counts. Results do not depend on it; it only costs time.
 */
tpcf_status tpcf_rebinned_count(tpcf_handle h, int64_t* h_out);

/*
 * Per-stage device time. With enable != 0 the handle records HIP events around
 * each stage it enqueues; tpcf_stage_times then returns, after tpcf_sync, the
 * summed milliseconds of the stages since the last reset and resets them:
 *  h_ms[0] grid build, [1] pair binning, [2] pair harmonics (a_lm),
 *  [3] contraction, [4] finalisation (3PCF and 2PCF multipoles), [5] 2PCF
 *  pair counts; h_launches[k] counts the launches timed.
 * Either output may be NULL; at most n entries are written.
 */
tpcf_status tpcf_set_timing(tpcf_handle h, int enable);
tpcf_status tpcf_stage_times(tpcf_handle h, int32_t n, double* h_ms, int64_t* h_launches);

#ifdef __cplusplus
}
#endif

#endif /* TPCF_H */
