/*
 * vpet_abc.h -- C ABI of the MI355X (gfx950) library for voxelwise ABC
 * rejection in dynamic PET kinetic modelling (vPET-ABC, arXiv 2603.14859).
 *
 * Per voxel the library draws kinetic parameters from a uniform prior box
 * (Alg. 1, lines 1-2), forward-simulates the frame-averaged time-activity curve
 * of a compartment model (Eq. (1)-(2); Alg. 1, line 3), scores every draw with
 * a noise-weighted distance to the observed curve (Alg. 1, line 4), keeps the
 * n = floor(N p) closest draws (Alg. 1, line 5 and the remark after it; the
 * fixed-budget variant of Sec. II-C) and reduces them to per-model posterior
 * means and variances and model probabilities (Eq. (6); Sec. II-D3; Ki per
 * accepted sample as in Sec. III-B2).
 *
 * Entry points: vpet_abc_infer (the whole path, independent draws per voxel;
 * vpet_abc_infer_noalloc is the same call without device allocation),
 * vpet_abc_simulate and vpet_abc_draws (single steps, for checking),
 * vpet_abc_bank_build + vpet_abc_infer_bank (Alg. 1 with one bank of draws
 * shared by every voxel), vpet_abc_stream_bank (the bank form over a volume in
 * a file), and the learned proposal vpet_proposal_* (not in the paper) whose
 * outputs drive importance-weighted draws in vpet_abc_infer.
 *
 * Conventions shared by every entry point
 *  - Every function returns a vpet_status and never throws or aborts.  On a
 *    status other than VPET_OK, vpet_abc_last_error() returns a message for the
 *    calling thread; nothing has been enqueued for VPET_E_ARG, VPET_E_MODEL,
 *    VPET_E_GRID and VPET_E_LIMIT.
 *  - "device" pointers are HIP device memory on the current device (the
 *    caller's hipSetDevice); "host" pointers are ordinary host memory that the
 *    library reads before the call returns.  The caller owns every buffer; the
 *    library writes only the out_* buffers it is given.
 *  - Device scratch that a call allocates in stream order comes from the
 *    device's default memory pool (hipMallocAsync); on first use of a device
 *    the library raises that pool's release threshold to 32 GiB, so that
 *    freed scratch is kept for the next call instead of being unmapped and
 *    mapped again.
 *  - Work is enqueued on `hip_stream` (a hipStream_t; NULL = the null stream)
 *    and the call returns without waiting.  Outputs are valid once the stream
 *    has reached that point.  Calls on different streams may overlap.
 *  - Time is in minutes, activity in any consistent unit (kBq/mL in the tests).
 *  - Time grid: nodes t_k = k * dt, k = 0..n_nodes-1.  The input function is
 *    given at the nodes and taken as linear between them.  Frame bounds
 *    frame_times[0..n_frames] must increase strictly and lie on nodes (to a
 *    relative 1e-6).
 *  - Parameter slots (stride VPET_PSTRIDE): 0 K1, 1 k2, 2 k3, 3 k4, 4 vB,
 *    5 Ki (derived, outputs only), 6-7 unused.  A model uses K1,k2,vB (1TCM),
 *    K1,k2,k3,vB (irreversible 2TCM, k4 = 0) or K1,k2,k3,k4,vB (reversible).
 *  - Draws are stratified by model: every model in model_id gets exactly
 *    n_draws draws per voxel; the global draw index of draw i of the model at
 *    list position m is g = m * n_draws + i.  Models are listed in bit order.
 *  - Draw (v, i) of list position m uses Philox4x32-10 (Salmon et al., SC'11)
 *    with key (seed low 32 bits, seed high 32 bits) and counter
 *    (i, v, 0, m << 16 | blk); parameter j of the model takes word j % 4 of
 *    block blk = j / 4 and becomes
 *        theta = fmaf((float)(hi - lo), (float)(word >> 8) * 2^-24, (float)lo).
 *    v is the global voxel index (voxel_offset + row).
 */
#ifndef VPET_ABC_H
#define VPET_ABC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    VPET_OK = 0,
    VPET_E_ARG = 1,    /* invalid argument (sizes, pointers, prior box, p)      */
    VPET_E_MODEL = 2,  /* unknown or empty model bitmask, or a model the call
                        * does not run                                          */
    VPET_E_GRID = 3,   /* frame bound off the grid, outside it, or not increasing */
    VPET_E_HIP = 4,    /* HIP runtime or launch failure                          */
    VPET_E_NOMEM = 5,  /* device or pinned-host allocation failed                */
    VPET_E_LIMIT = 6,  /* valid request beyond a documented capacity             */
    VPET_E_IO = 7      /* a file could not be opened, read or written            */
} vpet_status;

#define VPET_M_1TCM (1u << 0)     /* one-tissue model: K1 exp(-k2 t)                 */
#define VPET_M_2TCM_IRR (1u << 1) /* two-tissue, irreversible (k4 = 0), Eq. (1)-(2)   */
#define VPET_M_2TCM_REV (1u << 2) /* two-tissue, reversible, Eq. (1)-(2)              */
/* Reference-tissue models (Sec. II-A2): the input is the reference-region TAC
 * C_r, and Eq. (3)-(4) is read as the ODE C_t' = R1 C_r' + k2 C_r - kappa C_t,
 * kappa(t) = k2a + gamma g(t), C_t(0) = R1 C_r(0), with the activation
 * g(t) = s^alpha exp(alpha (1 - s)), s = (t - tD)/(tP - tD), zero up to tD
 * (peak 1 at tP).  lp-ntPET freezes kappa at each grid step's midpoint and
 * integrates the step exactly; MRTM is the gamma = 0 case, one exponential
 * exp(-k2a t) of amplitude k2 - R1 k2a plus the direct term R1 C_r.  The two
 * families cannot be mixed in one model_id (their inputs differ). */
#define VPET_M_MRTM (1u << 3)
#define VPET_M_LPNTPET (1u << 4)

#define VPET_PSTRIDE 8
#define VPET_SLOT_K1 0
#define VPET_SLOT_K2 1
#define VPET_SLOT_K3 2
#define VPET_SLOT_K4 3
#define VPET_SLOT_VB 4
#define VPET_SLOT_KI 5
/* Slots of the reference-tissue models (MRTM uses R1, k2, k2a).  The prior box
 * entry of tP is relative: tP is drawn in [tD + lo, hi] (lo > 0, tD_hi + lo <=
 * hi) as fmaf((float)hi - l, u, l), l = tD + (float)lo in fp32.  BP_ND =
 * k2 / k2a - 1 is reported in its slot per accepted sample. */
#define VPET_SLOT_R1 0
#define VPET_SLOT_RK2 1
#define VPET_SLOT_K2A 2
#define VPET_SLOT_GAMMA 3
#define VPET_SLOT_TD 4
#define VPET_SLOT_TP 5
#define VPET_SLOT_ALPHA 6
#define VPET_SLOT_BP 7

/* Capacities.  VPET_MAX_ACCEPT bounds n = floor(N p) (the accepted set of a
 * voxel is kept on chip); larger n returns VPET_E_LIMIT. */
#define VPET_MAX_ACCEPT 3968
#define VPET_MAX_NODES 16385
#define VPET_MAX_FRAMES 1024
#define VPET_BANK_MAX_FRAMES 48
#define VPET_BANK_MAX_ACCEPT 512
/* FP32 parameter blob of the learned proposal network (see
 * vpet_proposal_init): W1 [32][256], b1 [256], W2 [256][256], b2 [256],
 * W3 [256][96], b3 [96] (outputs 72..95 unused). */
#define VPET_PROPOSAL_NPARAM 98912
#define VPET_PROPOSAL_NOUT 96

typedef struct {
    float dt;         /* grid step (min), > 0                         */
    int32_t n_nodes;  /* K + 1 >= 2: input samples at t_k = k * dt     */
    int32_t n_frames; /* F >= 1                                        */
} vpet_grid;

/* Optional settings of vpet_abc_infer.  Zero-initialised = defaults. */
typedef struct {
    /* Decay constant (1/min) in the default weights; 0 -> ln 2 / 109.8 (18F). */
    double decay_lambda;
    /* device [V][F] caller weights w_vf >= 0 (inverse-variance sense); a
     * voxel with a negative or non-finite weight is invalid (NaN outputs,
     * like a non-finite observation).  NULL -> w_vf = dt_f exp(-lambda
     * tmid_f) / max(y_vf, floor * max_f y_vf), the inverse of the Sec. III-A1
     * noise variance with the unknown true curve replaced by the observation. */
    const float* weights;
    /* floor in the default weights as a fraction of max_f y_vf; 0 -> 0.01. */
    float weight_floor_frac;
    /* 0: d = sum_f w_f (y_f - x_f)^2 (default); 1: d = sum_f sqrt(w_f) |y_f - x_f|
     * (the L1 distance recommended in Sec. V, Conclusions and Limitations). */
    int32_t distance;
    /* Debug / parity outputs (device, may be NULL): accepted global draw
     * indices [V][n] and their fp32 distances [V][n] in ascending (d, g) order,
     * and the n-th smallest distance [V]. */
    int32_t* out_accept_idx;
    float* out_accept_dist;
    float* out_threshold;
    /* Global index of tacs row 0 (voxel chunking); row r is voxel
     * voxel_offset + r in the Philox counter. */
    int64_t voxel_offset;
    /* Waves cooperating on one voxel (1, 2 or 4); 0 = chosen from V. */
    int32_t waves_per_voxel;
    /* Shared-bank form only: bank rows in the pilot that sets each voxel's
     * candidate threshold; 0 = a default that lets about 4 n rows pass
     * (FP64 scan: the 16th smallest distance of ceil(4 N / n) rows; BF16
     * scan: the 16th smallest of 32 column minima of ceil(5.5 N / n) rows);
     * the pilot rows are spread evenly over the bank, which is ordered by
     * model. */
    int64_t bank_pilot;
    /* Shared-bank form only: how every (voxel, bank row) pair is screened.
     * 0 = auto (1 for L1, 2 for L2); 1 = FP64 distances on the vector ALUs;
     * 2 = the L2 distance as a voxels x rows x frames contraction on BF16
     * matrix cores (hi/lo split operands, FP32 accumulation, a per-pair error
     * bound), candidates re-ranked with exact FP64 distances.  Both give the
     * same accepted sets. */
    int32_t bank_scan;
    /* Shared-bank form only: host pointer; when set, the call brackets each
     * voxel chunk's scan kernel (the one that screens every (voxel, bank row)
     * pair) with HIP events on hip_stream, waits for them, and writes the
     * summed kernel time in milliseconds here.  Makes the call synchronous. */
    float* out_scan_ms;
    /* Shared-bank form only: host pointer; when set, receives the number of
     * voxels whose candidate list could not certify the accepted set and
     * that were redone by the exact pass over the whole bank.  Makes the call
     * synchronous. */
    int64_t* out_fallback_voxels;
    /* vpet_abc_infer only: device [n_voxels][VPET_PROPOSAL_NOUT] outputs of the
     * learned proposal network (vpet_proposal_forward) for each voxel.  When
     * set, the n_draws draws of each voxel come from its mixture instead of
     * the prior, draws outside the prior box are discarded, and the moments
     * are weighted by prior / proposal (importance-weighted ABC: the target is
     * unchanged).  Draw i of voxel v takes one Philox4x32-10 block, counter
     * (i, v, 2, 0), the seed as key: u0 = ((w0 & 255) | (w1 & 255) << 8 |
     * (w2 & 255) << 16) 2^-24 chooses the prior (u0 < share) or a mixture
     * component, and u_j = (w_j >> 8) 2^-24 (j = 0..3) give either the
     * uniform box draw or two Box-Muller pairs.  The irreversible 2TCM alone
     * (VPET_E_MODEL otherwise); model probability 1. */
    const float* proposal;
    /* device [n_voxels]: effective sample size (sum w)^2 / sum w^2 of each
     * voxel's accepted weights; needs proposal. */
    float* out_ess;
    /* With proposal: defensive prior share a in [0, 1].  The draws come from
     * a p + (1 - a) q (prior p, network mixture q): u0 < a draws uniformly
     * from the prior box, and every weight is p / (a p + (1 - a) q) <= 1 / a.
     * 0 = the network mixture alone. */
    double proposal_prior_share;
    /* With proposal: factor (> 0) on every component's sd; 0 -> 1. */
    double proposal_sd_scale;
    /* With proposal: device [n_voxels] fp32 thresholds h_v.  Of the n kept
     * draws, only those with fp32 distance <= h_v enter the moments, the
     * weights and the ESS: ABC with a given threshold (the indicator form of
     * Eq. (7)) instead of a given fraction.  The caller picks n large enough
     * that the n-th distance (out_threshold) exceeds h_v; otherwise the kept
     * draws are the n closest ones below h_v.  A voxel with no kept draw at or
     * below h_v (or h_v NaN) gets NaN moments, probability and ESS.  NULL =
     * every kept draw counts. */
    const float* accept_below;
} vpet_abc_opts;

/*
 * n = floor(n_total * accept_frac + 1e-6) (remark after Alg. 1; the 1e-6
 * absorbs products that land just below an integer).  Host-only.
 * Errors: VPET_E_ARG if n_total < 1, accept_frac outside (0, 1], n < 1 or
 * out_n is NULL.
 */
int vpet_abc_accept_count(int64_t n_total, double accept_frac, int64_t* out_n);

/*
 * Frame-averaged model curves for n parameter rows (Eq. (1)-(2), C_wb = C_p;
 * Alg. 1, line 3).  Each row is run in FP64 from its fp32 values; the frame
 * value is the trapezoid rule over the frame's nodes of the exact response to
 * the piecewise-linear input, divided by the frame length.
 *   model_id    exactly one VPET_M_* bit (any model)
 *   theta       device [n][VPET_PSTRIDE] fp32, slots as above (others ignored)
 *   input_fn    host [grid.n_nodes] fp32 (the reference TAC for MRTM, lp-ntPET)
 *   frame_times host [grid.n_frames + 1] fp32
 *   out_tacs    device [n][grid.n_frames] fp32
 * Errors: VPET_E_MODEL (not exactly one known bit), VPET_E_GRID, VPET_E_ARG
 * (n < 0, NULL pointers with n > 0, non-finite input), VPET_E_HIP.
 * n = 0 returns VPET_OK without enqueueing anything.
 */
int vpet_abc_simulate(uint32_t model_id, const float* theta, int64_t n, const float* input_fn,
                      const float* frame_times, vpet_grid grid, float* out_tacs, void* hip_stream);

/*
 * Voxelwise fixed-budget rejection ABC (Alg. 1).
 *   tacs          device [n_voxels][F] fp32 observed TACs
 *   frame_times   host [F + 1] fp32;  input_fn host [grid.n_nodes] fp32
 *   model_id      bitmask of the plasma-input VPET_M_* bits (1TCM, 2TCMs); M =
 *                 popcount, listed in bit order.  The reference-tissue models
 *                 run in the shared-bank form only (VPET_E_MODEL here): with a
 *                 subject-level reference TAC one bank serves every voxel.
 *   prior_box     host [M][VPET_PSTRIDE][2] FP64 (lo, hi) per slot; lo == hi
 *                 fixes a parameter.  Rate constants need lo >= 0, vB needs
 *                 0 <= lo and hi < 1; 2TCM models need k2_lo + k3_lo > 0 and the
 *                 reversible model k3_lo > 0 (distinct eigenvalues).
 *   n_draws       prior draws per model per voxel, M * n_draws < 2^32
 *   accept_frac   p in (0, 1]; n = floor(M n_draws p + 1e-6) in [1, VPET_MAX_ACCEPT]
 *   seed          Philox key
 *   out_moments   device [n_voxels][M][VPET_PSTRIDE][2] fp32: mean and
 *                 1/(cnt-1) variance of each slot over the accepted draws of
 *                 that model (cnt = 1 -> variance 0; cnt = 0 -> NaN); slot 5
 *                 is Ki = K1 k3 / (k2 + k3) for the 2TCM models; unused
 *                 slots are NaN.  Accumulated in FP64.
 *   out_model_prob device [n_voxels][M] fp32: cnt_m / n (Eq. (6)).
 *   opts          optional (NULL = defaults)
 * A voxel whose observed TAC has a non-finite value or max_f y <= 0 gets NaN
 * moments and probabilities (debug outputs: index -1, distance NaN).
 * The accepted set is the n smallest keys (fp32(d), g): ties in fp32 distance
 * go to the lower global draw index.
 * Errors: VPET_E_ARG, VPET_E_MODEL, VPET_E_GRID, VPET_E_LIMIT (see above),
 * VPET_E_NOMEM, VPET_E_HIP.  n_voxels = 0 returns VPET_OK with no launch.
 */
int vpet_abc_infer(const float* tacs, int64_t n_voxels, const float* frame_times,
                   const float* input_fn, vpet_grid grid, uint32_t model_id,
                   const double* prior_box, int64_t n_draws, double accept_frac, uint64_t seed,
                   float* out_moments, float* out_model_prob, const vpet_abc_opts* opts,
                   void* hip_stream);

/*
 * vpet_abc_infer for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same arguments, kernels and results, and no hipMalloc, hipFree or other
 * allocating routine.  The call's draw-independent tables (input nodes,
 * per-frame sums and lengths) are written in stream order into one 256 KB
 * device array that the library holds on every GPU it runs on until the
 * process ends; the largest grid (VPET_MAX_NODES nodes, VPET_MAX_FRAMES
 * frames) needs about 165 KB, and a request beyond 256 KB returns
 * VPET_E_LIMIT.  Every call on a GPU shares that array, which keeps the last
 * call's tables: calls on one stream are ordered, but calls that overlap on
 * one GPU (other streams, other host threads) race -- the caller orders them.
 * Errors: those of vpet_abc_infer except VPET_E_NOMEM.
 */
int vpet_abc_infer_noalloc(const float* tacs, int64_t n_voxels, const float* frame_times,
                           const float* input_fn, vpet_grid grid, uint32_t model_id,
                           const double* prior_box, int64_t n_draws, double accept_frac, uint64_t seed,
                           float* out_moments, float* out_model_prob, const vpet_abc_opts* opts,
                           void* hip_stream);

/*
 * The prior draws themselves (Alg. 1, lines 1-2), for checking and for
 * re-deriving accepted samples.  For each of `count` triples (voxel[j],
 * draw[j], model_pos[j]) (device int64, int64, int32; voxel is the global
 * voxel index, model_pos the list position in model_id) writes the Philox
 * words of the draw (device [count][8] u32, block-major, unused words 0) and
 * theta (device [count][VPET_PSTRIDE] fp32, unused slots NaN).
 * Errors: VPET_E_MODEL, VPET_E_ARG (prior box as for infer, NULL pointers with
 * count > 0), VPET_E_HIP.  Out-of-range model_pos entries yield NaN theta.
 */
int vpet_abc_draws(uint32_t model_id, const double* prior_box, uint64_t seed,
                   const int64_t* voxel, const int64_t* draw, const int32_t* model_pos,
                   int64_t count, uint32_t* out_words, float* out_theta, void* hip_stream);

/*
 * Shared-bank form (Alg. 1 as printed: lines 1-3 are done once and the bank
 * of draws and curves serves every voxel).  Bank draw i of list position m is
 * the Philox draw of counter (i, 0, 1, m << 16 | blk) -- stream 1, no voxel
 * index -- so a bank is a function of (model_id, prior_box, n_draws, seed,
 * grid) only and may be reused across calls and voxel chunks.  Every model,
 * including the reference-tissue ones (input_fn = reference TAC), runs here;
 * the moments of the reference-tissue models carry BP_ND in slot 7.
 *
 * vpet_abc_bank_ld(F): row stride (frames rounded up to a multiple of 8) of the
 * bank curves.  Host-only; 0 for F <= 0.
 *
 * vpet_abc_bank_build writes
 *   out_theta  device [M * n_draws][VPET_PSTRIDE] fp32 (unused slots NaN)
 *   out_x      device [M * n_draws][vpet_abc_bank_ld(F)] FP64 frame averages
 *              (the same forward model as vpet_abc_simulate; padding 0)
 * Errors: as vpet_abc_infer; VPET_E_LIMIT if F > VPET_BANK_MAX_FRAMES.
 */
int vpet_abc_bank_ld(int32_t n_frames);
int vpet_abc_bank_build(uint32_t model_id, const double* prior_box, int64_t n_draws, uint64_t seed,
                        const float* input_fn, const float* frame_times, vpet_grid grid, float* out_theta,
                        double* out_x, void* hip_stream);

/*
 * Fixed-budget rejection ABC of every voxel against one bank (Alg. 1, lines
 * 4-5, and the summaries of vpet_abc_infer).  model_id and n_draws describe
 * the bank (bank_theta, bank_x as written by vpet_abc_bank_build on the same
 * grid); frame_times and grid give the frames (the input function is not
 * needed).  Distances are FP64; the accepted set is the n smallest keys
 * (fp32(d), g), n = floor(M n_draws p + 1e-6) <= VPET_BANK_MAX_ACCEPT.
 * opts: weights, weight_floor_frac, decay_lambda, distance, the debug outputs,
 * bank_pilot and bank_scan are honoured; voxel_offset and waves_per_voxel do
 * not apply.  Whatever the scan, the accepted set is the exact one: a voxel
 * whose candidate list cannot prove it holds the n smallest keys is redone
 * by an exact pass over the whole bank.
 * Device scratch (a candidate list of 8 n keys, or 16 n bank rows for the
 * BF16 scan, per voxel, in voxel chunks of at most 4 GiB; the BF16 operands,
 * 8 M n_draws ld bytes) is allocated and freed in stream order.
 * Errors: VPET_E_ARG, VPET_E_MODEL, VPET_E_GRID, VPET_E_LIMIT, VPET_E_NOMEM,
 * VPET_E_HIP.
 */
int vpet_abc_infer_bank(const float* tacs, int64_t n_voxels, const float* frame_times, vpet_grid grid,
                        uint32_t model_id, int64_t n_draws, double accept_frac, const float* bank_theta,
                        const double* bank_x, float* out_moments, float* out_model_prob,
                        const vpet_abc_opts* opts, void* hip_stream);

/*
 * Shared-bank form with a learned proposal (not in the paper: the bank of
 * Alg. 1, lines 1-3, drawn from a proposal instead of the prior, with every
 * bank row weighted by prior / proposal so that each voxel's ABC target is
 * unchanged).  The voxels are grouped by the posterior that the network
 * (vpet_proposal_forward) gives for them, and each group gets its own bank:
 *  1. cells: each voxel's mixture over z = log theta (a head over `dims`
 *     parameters) has mean m_j and second moment s_j per parameter; cell
 *     coordinate j is floor(bins (exp(m_j) - lo_j) / (hi_j - lo_j)) clamped to
 *     [0, bins - 1] over the prior box of the head's parameters (the box of
 *     the last model listed), and the cells are numbered along a serpentine
 *     walk (coordinate j runs backwards when the number of the coordinates
 *     before it is odd), so that consecutive cells are neighbours; a voxel
 *     whose observation is invalid (as in vpet_abc_infer) comes last;
 *  2. groups: the voxels sorted by cell (ties by voxel index) are cut into
 *     groups of group_voxels consecutive voxels (G = ceil(n_voxels /
 *     group_voxels) groups);
 *  3. proposals: group g's Gaussian has, per head parameter, the mean mu_j =
 *     avg m_j and the sd sqrt(avg s_j - mu_j^2) * sd_scale over its valid
 *     members (FP64 sums, stored in fp32), mixed with the prior with the
 *     defensive share a = prior_share: the proposal is a p + (1 - a) q_g;
 *  4. banks: n_draws rows per model per group; row i of list position m of
 *     group g uses Philox4x32-10 counters (i, G0 + g, 3, m << 16) and (i,
 *     G0 + g, 3, m << 16 | 1) (G0 = first_group; the second counter only for
 *     five-parameter models), the seed as
 *     key; u0 = ((w0 & 255) | (w1 & 255) << 8 | (w2 & 255) << 16) 2^-24 < a
 *     (or a group without valid members) draws every parameter uniformly,
 *     theta_p = fp32(lo_p + u_p wid_p) (lo_p, wid_p = hi_p - lo_p in fp32);
 *     otherwise theta_p = fp32(exp(mu_d + sd_d n_p)) for each parameter with
 *     a head parameter d (a draw outside the box gets weight 0) and a
 *     uniform draw from u_6 for k4 under a four-parameter head; u_p = (w_p >>
 *     8) 2^-24 (p < 4), u_4, u_5, u_6 = (v0, v1, v2 >> 8) 2^-24, normals n_2q,
 *     n_2q+1 = r cos, r sin (2 pi u_2q+1), r = sqrt(-2 ln(u_2q + 2^-24));
 *     log w = -log(a + (1 - a) e^L), L = sum over the head's parameters of
 *     log N(z_p; mu_d, sd_d) - z_p + log wid_p (z_p = log theta_p for a
 *     uniform draw); every row is simulated as in vpet_abc_bank_build;
 *  5. each voxel runs the bank form of vpet_abc_infer_bank against its
 *     group's bank (n = floor(M n_draws p + 1e-6) closest rows, the exact
 *     accepted set whatever the scan), and the accepted rows count with their
 *     weights: per model m, probability sum_m w / sum w and weighted means
 *     and variances sum w (t - mean)^2 / sum w (Ki in slot 5; FP64).
 *   model_id      VPET_M_2TCM_IRR and/or VPET_M_2TCM_REV.  A four-parameter
 *                 head (K1, k2, k3, vB) drives both (k4 of the reversible
 *                 model then comes from the prior); a five-parameter head
 *                 (K1, k2, k3, k4, vB) drives the irreversible model through
 *                 its four shared parameters.
 *   proposal      device [n_voxels][VPET_PROPOSAL_NOUT] network outputs
 *   groups        the grouping (below); n_draws per model per group
 *   opts          weights, weight_floor_frac, decay_lambda, distance, the
 *                 debug outputs (out_accept_idx holds rows of the group's bank
 *                 as numbered in out_bank_theta), bank_pilot, bank_scan,
 *                 out_scan_ms, out_fallback_voxels, out_ess and accept_below
 *                 are honoured; proposal, voxel_offset and waves_per_voxel
 *                 must be unset.
 * Device scratch (the grouping, about 40 + 4 F bytes per voxel; the banks of
 * one chunk of whole groups within 16 GiB and its candidate lists within 4
 * GiB) is allocated and freed in stream order.
 * Errors: VPET_E_ARG, VPET_E_MODEL, VPET_E_GRID, VPET_E_LIMIT (bins^dims >
 * 4096, n > VPET_BANK_MAX_ACCEPT, F > VPET_BANK_MAX_FRAMES, more than 2^31 - 1
 * voxels), VPET_E_NOMEM, VPET_E_HIP.
 */
typedef struct {
    int32_t dims;          /* 4 or 5: the network head (vpet_proposal_train)         */
    int32_t bins;          /* cells per parameter, >= 1, bins^dims <= 4096            */
    int32_t group_voxels;  /* voxels per group: a positive multiple of 256            */
    double prior_share;    /* defensive share a in [0, 1]                             */
    double sd_scale;       /* factor (> 0) on each group's sd; 0 -> 1                 */
    int64_t first_group;   /* added to the group index g in the Philox counters       */
    int32_t* out_group;    /* device [n_voxels] group of each voxel, or NULL          */
    float* out_bank_theta; /* device [G][M n_draws][VPET_PSTRIDE] bank draws, or NULL */
    double* out_bank_logw; /* device [G][M n_draws] log weights, or NULL              */
} vpet_bank_groups;

int vpet_abc_infer_bank_learned(const float* tacs, int64_t n_voxels, const float* frame_times,
                                const float* input_fn, vpet_grid grid, uint32_t model_id,
                                const double* prior_box, const float* proposal,
                                const vpet_bank_groups* groups, int64_t n_draws, double accept_frac,
                                uint64_t seed, float* out_moments, float* out_model_prob,
                                const vpet_abc_opts* opts, void* hip_stream);

/*
 * The BF16 contraction scan's own values, for checking its error bound (the
 * screening step of vpet_abc_infer_bank with bank_scan = 2, Alg. 1 line 4 as
 * a contraction).  With A_v = [-2 w y, w] (FP64 from the voxel's fp32 curve
 * and weights, as in vpet_abc_infer_bank) and B_g = [x_g, x_g^2], both split
 * into bf16 hi + lo parts, the scan computes S_vg ~ sum_k A_vk B_gk as
 * hi*hi + hi*lo + lo*hi on the matrix cores with FP32 accumulation, and
 * d_vg = a_v + sum_k A_vk B_gk exactly (a_v = sum_f w y^2).  This call runs
 * the operand kernels and the scan kernel itself with a candidate test that
 * admits every pair, and writes
 *   out_s  device [n_voxels][n_rows] fp32: S_vg (NaN for an invalid voxel)
 *   out_a  device [n_voxels] FP64: a_v (NaN for an invalid voxel, -inf for a
 *          voxel with a negative caller weight)
 * for bank_x device [n_rows][vpet_abc_bank_ld(F)] FP64 rows.  The scan's
 * candidate test relies on |S_vg - sum_k A_vk B_gk| <= m E_vg with
 * E_vg = sum_k |A_vk| |B_gk| and m = 2 (3 2^-16 + 3 K 2^-24), K = 2 ld.
 * opts: weights, weight_floor_frac and decay_lambda are honoured.
 * 1 <= n_rows <= 4096 and n_voxels <= 65536 (VPET_E_LIMIT beyond).  Device
 * scratch is allocated and freed in stream order.
 * Errors: VPET_E_ARG, VPET_E_GRID, VPET_E_LIMIT, VPET_E_NOMEM, VPET_E_HIP.
 */
int vpet_abc_bank_screen(const float* tacs, int64_t n_voxels, const float* frame_times, vpet_grid grid,
                         const double* bank_x, int64_t n_rows, const vpet_abc_opts* opts, float* out_s,
                         double* out_a, void* hip_stream);

/*
 * Streamed shared-bank inference of a volume stored in a file (total-body
 * scale; the whole-volume study of Sec. III-B2).  The observed TACs are read
 * chunk by chunk from tacs_path (raw little-endian fp32, [n_voxels][F]
 * row-major, F = grid.n_frames); while chunk c is screened on the GPU, chunk
 * c+1 is read and copied in and the outputs of chunk c-1 are written (by a
 * host thread that the call starts and joins before it returns) to
 *   <out_prefix>.moments   [n_voxels][M][VPET_PSTRIDE][2] fp32
 *   <out_prefix>.prob      [n_voxels][M] fp32
 * at their voxel offsets.  After the outputs of a chunk are on disk,
 * <out_prefix>.progress (one text line: the run's shape and the number of
 * completed chunks, replaced atomically) is updated, so a run that stops --
 * killed, or by max_chunks -- continues with resume != 0 from the first
 * incomplete chunk; resume == 0 starts over.
 *   model_id, n_draws, accept_frac, bank_theta, bank_x: as vpet_abc_infer_bank
 *   chunk_voxels  voxels per chunk, >= 1 (pinned host and device buffers hold
 *                 two chunks of input and output)
 *   max_chunks    process at most this many chunks in this call (0 = all)
 *   out_done      host, optional: completed chunks after the call
 *   opts          as vpet_abc_infer_bank, except that caller weights, the
 *                 debug outputs and the timing/fallback reports are refused
 *                 (VPET_E_ARG); NULL = defaults
 * The call returns when the processed chunks are on disk (synchronous); it
 * uses hip_stream for the kernels and one internal stream for the copies in.
 * Each voxel's outputs are those of vpet_abc_infer_bank on the same data.
 * Errors: those of vpet_abc_infer_bank; VPET_E_IO for files (missing or short
 * input, unwritable outputs); VPET_E_ARG for a progress file of another run's
 * shape when resuming.
 */
int vpet_abc_stream_bank(const char* tacs_path, int64_t n_voxels, const float* frame_times, vpet_grid grid,
                         uint32_t model_id, int64_t n_draws, double accept_frac, const float* bank_theta,
                         const double* bank_x, int64_t chunk_voxels, const char* out_prefix, int32_t resume,
                         int64_t max_chunks, const vpet_abc_opts* opts, int64_t* out_done, void* hip_stream);

/*
 * vpet_abc_stream_bank with a learned proposal: the same streaming (file in,
 * two chunks in flight, outputs and progress on disk, resume), where each
 * chunk runs the network (vpet_proposal_forward with params) and then
 * vpet_abc_infer_bank_learned on the chunk's voxels; the grouping is made
 * within each chunk (a voxel's outputs depend on the chunk it is in, which
 * chunk_voxels fixes), and chunk c numbers its groups from first_group +
 * c ceil(chunk_voxels / group_voxels) in the Philox counters.  model_id, prior_box, groups (the out_* members must
 * be NULL), n_draws, accept_frac and seed as vpet_abc_infer_bank_learned;
 * opts as vpet_abc_stream_bank (out_ess and accept_below refused).  F <= 32.
 * The progress file names this kind of run, so a resume does not continue a
 * prior-bank run or the reverse.  Device buffers of one chunk's network
 * outputs are allocated and freed by the call, which returns when the
 * processed chunks are on disk.
 * Errors: those of vpet_abc_stream_bank and vpet_abc_infer_bank_learned.
 */
int vpet_abc_stream_bank_learned(const char* tacs_path, int64_t n_voxels, const float* frame_times,
                                 const float* input_fn, vpet_grid grid, uint32_t model_id,
                                 const double* prior_box, const float* params, const vpet_bank_groups* groups,
                                 int64_t n_draws, double accept_frac, uint64_t seed, int64_t chunk_voxels,
                                 const char* out_prefix, int32_t resume, int64_t max_chunks,
                                 const vpet_abc_opts* opts, int64_t* out_done, void* hip_stream);

/*
 * Learned proposal for importance-weighted ABC (not in the paper: an
 * amortised proposal for the prior draws of Alg. 1, lines 1-2; the ABC
 * target is unchanged because accepted draws carry the weight prior /
 * proposal).  The network maps features x_f = log1p(max(y_f, 0)) of a TAC
 * (zero-padded to 32 inputs; F <= 32, VPET_E_LIMIT otherwise) through
 * relu(x W1 + b1), relu(h1 W2 + b2), h2 W3 + b3 to 72 outputs: 8 mixture
 * logits, 8 x 4 means and 8 x 4 raw scales of a Gaussian mixture over
 * z = log(K1, k2, k3, vB) of the irreversible 2TCM, with log sd = -6 +
 * 8 sigmoid(raw).  The products run on BF16 matrix cores: each fp32 operand
 * is split into bf16 hi + lo and three products are accumulated in FP32
 * (about 3 * 2^-16 relative error per term; FP32 master weights); params is
 * the VPET_PROPOSAL_NPARAM-float blob laid out as documented at that
 * constant.  All pointers are device pointers
 * unless stated; every call is asynchronous on hip_stream unless stated.
 */

/* He-normal weights (sd sqrt(2 / fan_in), the output layer sqrt(1 / fan_in))
 * and zero biases into params, normals from Philox stream 5 keyed by seed.
 * Errors: VPET_E_ARG (NULL params), VPET_E_HIP. */
int vpet_proposal_init(float* params, uint64_t seed, void* hip_stream);

/* out [n][VPET_PROPOSAL_NOUT] = network outputs of the TACs tacs [n][n_frames]
 * (fp32 row-major); columns 72..95 are padding.  Scratch for at most 2^17
 * rows at a time is allocated and freed in stream order.
 * Errors: VPET_E_ARG, VPET_E_LIMIT (n_frames outside 1..32), VPET_E_NOMEM,
 * VPET_E_HIP. */
int vpet_proposal_forward(const float* params, const float* tacs, int64_t n, int32_t n_frames, float* out,
                          void* hip_stream);

/* Heads.  The outputs are read as a mixture over D = dims parameters:
 * dims = 4 (the layout above): z = log(K1, k2, k3, vB), outputs 0..71;
 * dims = 5: z = log(K1, k2, k3, k4, vB), outputs 0..7 logits, 8..47 means
 * (component c, parameter j at 8 + 5 c + j), 48..87 raw scales (48 + 5 c +
 * j).  A five-parameter head is trained on reversible-2TCM draws (k4 in slot
 * 3) and drives the reversible model of vpet_abc_infer_bank_learned, and the
 * irreversible one through the marginal of its other four parameters. */

/* Training loss and its gradient for one batch: loss[0] = mean over the n
 * rows of -log q(z | tacs), z = log(max(theta, 1e-6)) of the head's slots
 * (K1, k2, k3, vB for dims = 4; K1, k2, k3, k4, vB for dims = 5) of theta
 * [n][VPET_PSTRIDE] (fp32, the bank layout); grad [VPET_PROPOSAL_NPARAM] is
 * overwritten with d loss / d params (the unused outputs get zero gradient).
 * 1 <= n <= 2^20.  Errors: VPET_E_ARG (also dims not 4 or 5), VPET_E_LIMIT,
 * VPET_E_NOMEM, VPET_E_HIP. */
int vpet_proposal_loss_grad(const float* params, const float* tacs, const float* theta, int64_t n,
                            int32_t n_frames, int32_t dims, float* grad, float* loss, void* hip_stream);

/* `steps` Adam steps (beta 0.9, 0.999, eps 1e-8; the step size follows a
 * cosine decay from learning_rate at the first step towards 0) on params, a
 * head over `dims` parameters (4 or 5, as vpet_proposal_loss_grad), trained
 * on the shared bank of vpet_abc_bank_build (bank_theta, bank_x with n_bank
 * rows of one irreversible 2TCM bank for dims = 4, one reversible 2TCM bank
 * for dims = 5): step t takes `batch`
 * consecutive rows of a seeded affine permutation of the bank (a new one per
 * pass) and adds fresh Gaussian noise of variance
 * noise_level e^{decay_lambda tmid_f} max(x_f, 0) / dt_f to each frame
 * (Sec. III-A1 noise; Philox stream 4 keyed by seed); frame_times is host
 * [n_frames + 1].  out_loss (host, optional, [steps]) receives each step's
 * batch loss, which makes the call synchronous.  Scratch (Adam moments, one
 * batch of activations and the partial sums of the weight-gradient products,
 * which are split over the batch rows and added in a fixed order, so training
 * is deterministic) is allocated and freed in stream order.
 * Errors: VPET_E_ARG, VPET_E_GRID (frame bounds), VPET_E_LIMIT, VPET_E_NOMEM,
 * VPET_E_HIP. */
int vpet_proposal_train(float* params, const float* bank_theta, const double* bank_x, int64_t n_bank,
                        const float* frame_times, int32_t n_frames, int32_t dims, double noise_level,
                        double decay_lambda, int64_t steps, int32_t batch, float learning_rate, uint64_t seed,
                        float* out_loss, void* hip_stream);

/* Message for the calling thread's last non-OK status ("" if none). */
const char* vpet_abc_last_error(void);

/* Library version, major * 10000 + minor * 100 + patch. */
int vpet_abc_version(void);

#ifdef __cplusplus
}
#endif

#endif /* VPET_ABC_H */
