/*
 * vpet_oracle.c -- plain, slow, FP64 CPU oracle for voxelwise ABC rejection
 * (vPET-ABC, arXiv 2603.14859).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the reference that the GPU library is
 * checked against.  Only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark may load it.  It shares no code, header, table or
 * constant generator with the HIP library; both are written independently from
 * the paper and from the numerics readings listed beside each function.
 *
 * Everything is done the obvious way: one voxel at a time, one draw at a time,
 * FP64 throughout, a library sort for the selection, two-pass moments.  The only
 * concession to speed is an optional OpenMP loop over voxels (voxels are
 * independent; the result does not depend on the thread count).
 *
 * Paper passages followed (section / equation / algorithm / table):
 *   - 2TCM ODE and measured activity: Sec. II-A1, Eq. (1)-(2).
 *   - Posterior / model posterior: Sec. II-B, Eq. (5)-(6).
 *   - Fixed-budget rejection ABC: Sec. II-C ("vPET-ABC" paragraph) and Alg. 1;
 *     n = floor(N p): the remark that follows Alg. 1.
 *   - Noise model (used for the default discrepancy weights): Sec. III-A1.
 *   - Posterior mean as point estimate: Sec. II-D3.
 *   - Preferred model (> 50 %) and Ki = K1 k3 / (k2 + k3) per accepted sample:
 *     Sec. III-B2 (TB-PET study).
 *   - Counter-based generator: Philox4x32-10 of Salmon, Moraes, Dror and Shaw,
 *     "Parallel random numbers: as easy as 1, 2, 3", SC'11.
 *   - Reference-tissue models: lp-ntPET, Eq. (3)-(4) (Sec. II-A2); MRTM is its
 *     gamma = 0 case; the activation g(t) is the gamma variate of the lp-ntPET
 *     literature the section cites (peak 1 at t_P).
 *
 * Readings where the paper is silent (each is one line of the numerics spec):
 *   R1 draws: counter (i, v, stream, m<<16 | blk), key = seed; word -> u =
 *      (w >> 8) * 2^-24; theta_f32 = fmaf((float)(hi-lo), u, (float)lo).
 *   R2 simulation: input linearly interpolated between grid nodes t_k = k h;
 *      each exponential convolved exactly over every step; frame value =
 *      trapezoid of the node TAC over the frame's nodes / frame length.
 *   R3 weights: w_f = dt_f exp(-lambda tmid_f) / max(y_f, floor * max_f y_f).
 *   R4 distance: weighted L2 (default) or weighted L1 with sqrt(w_f).
 *   R5 selection: keep the n smallest (d, g); ties go to the lower index g.
 *   R6 models: stratified, exactly n_draws per model; g = m n_draws + i.
 *   R7 variance: 1/(cnt-1); cnt = 1 -> 0; cnt = 0 -> NaN (and prob 0).
 *   R12 reference-tissue models: the input is the reference TAC C_r, linear
 *      between nodes.  Eq. (3)-(4) are the ODE C_t' = R1 C_r' + k2 C_r - kappa C_t,
 *      kappa(t) = k2a + gamma g(t), C_t(0) = R1 C_r(0); with C_t = R1 C_r + z,
 *      z' = (k2 - R1 kappa) C_r - kappa z.  MRTM (gamma = 0) is one exponential
 *      exp(-k2a t) of amplitude k2 - R1 k2a plus the direct term R1 C_r.  For
 *      lp-ntPET kappa is frozen at each step's midpoint and the step is then
 *      integrated exactly (the R2 step weights with rate kappa).
 *      g(t) = s^alpha exp(alpha (1 - s)), s = (t - tD)/(tP - tD), for t > tD.
 *   R13 lp-ntPET draws: the t_P box is relative to the drawn t_D:
 *      lo = tD + box_lo (fp32), t_P = fmaf((float)box_hi - lo, u, lo).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------------- */
/* Model identifiers and canonical parameter slots.                          */
/* ------------------------------------------------------------------------- */
#define ORA_M_1TCM 1u
#define ORA_M_2TCM_IRR 2u
#define ORA_M_2TCM_REV 4u
#define ORA_M_MRTM 8u
#define ORA_M_LPNT 16u
#define ORA_NSLOT 8 /* K1, k2, k3, k4, vB, Ki, unused, unused */
#define SLOT_K1 0
#define SLOT_K2 1
#define SLOT_K3 2
#define SLOT_K4 3
#define SLOT_VB 4
#define SLOT_KI 5
/* reference-tissue models: R1, k2, k2a, gamma, tD, tP, alpha, BP_ND = k2/k2a - 1 */
#define SLOT_R1 0
#define SLOT_RK2 1
#define SLOT_K2A 2
#define SLOT_GAMMA 3
#define SLOT_TD 4
#define SLOT_TP 5
#define SLOT_ALPHA 6
#define SLOT_BP 7

/* The slots a model draws, in the order its Philox words are consumed. */
static int model_params(uint32_t model, int slots[8]) {
    if (model == ORA_M_1TCM) {
        slots[0] = SLOT_K1; slots[1] = SLOT_K2; slots[2] = SLOT_VB;
        return 3;
    }
    if (model == ORA_M_2TCM_IRR) {
        slots[0] = SLOT_K1; slots[1] = SLOT_K2; slots[2] = SLOT_K3; slots[3] = SLOT_VB;
        return 4;
    }
    if (model == ORA_M_2TCM_REV) {
        slots[0] = SLOT_K1; slots[1] = SLOT_K2; slots[2] = SLOT_K3; slots[3] = SLOT_K4;
        slots[4] = SLOT_VB;
        return 5;
    }
    if (model == ORA_M_MRTM) {
        slots[0] = SLOT_R1; slots[1] = SLOT_RK2; slots[2] = SLOT_K2A;
        return 3;
    }
    if (model == ORA_M_LPNT) {
        for (int j = 0; j < 7; ++j) slots[j] = j; /* R1, k2, k2a, gamma, tD, tP, alpha */
        return 7;
    }
    return 0;
}

/* ------------------------------------------------------------------------- */
/* Philox4x32-10 (Salmon et al., SC'11).                                     */
/* One round: two 32x32->64 products of the round multipliers with words 0    */
/* and 2; the high halves are xor-ed with the other words and the key, the    */
/* low halves move into the odd positions.  The key is advanced by the two   */
/* Weyl constants between rounds.                                            */
/* ------------------------------------------------------------------------- */
void ora_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
    const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
    const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
    uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int r = 0; r < 10; ++r) {
        if (r > 0) {
            k0 += W0;
            k1 += W1;
        }
        uint64_t p0 = (uint64_t)M0 * (uint64_t)x0;
        uint64_t p1 = (uint64_t)M1 * (uint64_t)x2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ x1 ^ k0;
        uint32_t n2 = hi0 ^ x3 ^ k1;
        x0 = n0;
        x1 = lo1;
        x2 = n2;
        x3 = lo0;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/* Vectorised helper for tests: n counters [n][4] -> words [n][4]. */
void ora_philox_batch(const uint32_t* ctr, int64_t n, uint64_t seed, uint32_t* out) {
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    for (int64_t j = 0; j < n; ++j) ora_philox4x32_10(ctr + 4 * j, key, out + 4 * j);
}

/* 24 high bits of a word as a float in [0, 1): exact in fp32 and fp64. */
static float word_to_unit(uint32_t w) { return (float)(w >> 8) * (1.0f / 16777216.0f); }

/* Draw the parameters of model `model` (position m in the call's model list)
 * for voxel v, draw i.  box is the model's [8][2] (lo, hi) prior box.
 * theta gets the fp32 draw in canonical slots (unused slots NaN); words, if not
 * NULL, receives the Philox words ([2][4], block-major). Alg. 1, lines 1-2. */
void ora_draw(uint32_t model, const double* box, uint64_t seed, uint64_t v, uint64_t i,
              uint32_t m, uint32_t stream, float* theta, uint32_t* words, float* u_out) {
    int slots[8];
    int np = model_params(model, slots);
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t w[8] = {0};
    int nblk = (np + 3) / 4;
    for (int blk = 0; blk < nblk; ++blk) {
        uint32_t ctr[4] = {(uint32_t)i, (uint32_t)v, stream, (m << 16) | (uint32_t)blk};
        ora_philox4x32_10(ctr, key, w + 4 * blk);
    }
    for (int s = 0; s < ORA_NSLOT; ++s) theta[s] = NAN;
    for (int j = 0; j < np; ++j) {
        int s = slots[j];
        double lo = box[2 * s], hi = box[2 * s + 1];
        float lo_f = (float)lo;
        float wid_f = (float)(hi - lo);
        if (model == ORA_M_LPNT && s == SLOT_TP) { /* R13: t_P in [tD + lo, hi] */
            lo_f = theta[SLOT_TD] + (float)lo;
            wid_f = (float)hi - lo_f;
        }
        float u = word_to_unit(w[j]);
        theta[s] = fmaf(wid_f, u, lo_f);
        if (u_out) u_out[j] = u;
    }
    if (words) memcpy(words, w, sizeof(uint32_t) * 4 * (size_t)nblk);
}

/* Batch version for tests: n (v, i, m) triples. models[m] is the model bit
 * of list position m; boxes is [M][8][2]. */
void ora_draw_batch(const uint32_t* models, const double* boxes, uint64_t seed,
                    const int64_t* vv, const int64_t* ii, const int32_t* mm, int64_t n,
                    uint32_t stream, float* theta, uint32_t* words, float* u) {
    for (int64_t j = 0; j < n; ++j) {
        uint32_t m = (uint32_t)mm[j];
        ora_draw(models[m], boxes + (size_t)m * 16, seed, (uint64_t)vv[j], (uint64_t)ii[j], m,
                 stream, theta + 8 * j, words + 8 * j, u + 8 * j);
    }
}

/* ------------------------------------------------------------------------- */
/* Convolution of one exponential kernel exp(-beta t) with the input.        */
/* Reading R2: between nodes the input is the straight line through          */
/* (t_k, C_k) and (t_{k+1}, C_{k+1}); integrating the ODE  I' = -beta I + C   */
/* exactly over one step gives                                               */
/*   I_{k+1} = exp(-x) I_k + a C_k + b C_{k+1},   x = beta h,                */
/*   a = h (1 - (1 + x) e^{-x}) / x^2,   b = h (e^{-x} - 1 + x) / x^2.        */
/* For x < 0.1 both are evaluated by their Taylor series (x -> 0 gives the   */
/* trapezoid rule a = b = h/2, which is the beta = 0 case).                  */
/* ------------------------------------------------------------------------- */
void ora_step_coeffs(double beta, double h, double* e, double* a, double* b) {
    double x = beta * h;
    *e = exp(-x);
    if (x < 0.1) {
        /* a/h = sum_{m>=2} (-1)^m (m-1)/m! x^{m-2};  b/h = sum_{m>=2} (-1)^m x^{m-2}/m!
         * (the closed forms lose about eps/x^2 to cancellation; below x = 0.1 the
         * series, truncated after m = 12, is accurate to ~1e-19). */
        double sa = 0.0, sb = 0.0, xp = 1.0, fact = 2.0;
        for (int m = 2; m <= 12; ++m) {
            double sign = (m % 2 == 0) ? 1.0 : -1.0;
            sa += sign * (double)(m - 1) / fact * xp;
            sb += sign / fact * xp;
            xp *= x;
            fact *= (double)(m + 1);
        }
        *a = h * sa;
        *b = h * sb;
    } else {
        *a = h * (1.0 - (1.0 + x) * exp(-x)) / (x * x);
        *b = h * (exp(-x) - 1.0 + x) / (x * x);
    }
}

/* I_k for k = 0..K (I_0 = 0). */
void ora_convolve_exp(double beta, const double* cp, int K, double h, double* out) {
    double e, a, b;
    ora_step_coeffs(beta, h, &e, &a, &b);
    out[0] = 0.0;
    for (int k = 0; k < K; ++k) out[k + 1] = e * out[k] + a * cp[k] + b * cp[k + 1];
}

/* ------------------------------------------------------------------------- */
/* Impulse response of each model as a sum of exponentials A_j exp(-rate_j t) */
/* so that the tissue activity C_f + C_m = sum_j A_j (exp(-rate_j t) * C_p). */
/* Eq. (1): the 2TCM is linear with constant coefficients; its impulse        */
/* response for C_f + C_m is K1 (s + k3 + k4) / (s^2 + (k2+k3+k4) s + k2 k4)   */
/* in Laplace form, whose poles are -alpha_1, -alpha_2.                       */
/* Returns the number of terms (<= 2).                                        */
/* ------------------------------------------------------------------------- */
int ora_exp_terms(uint32_t model, const double* th, double rate[2], double amp[2]) {
    double K1 = th[SLOT_K1], k2 = th[SLOT_K2];
    if (model == ORA_M_1TCM) {
        rate[0] = k2;
        amp[0] = K1;
        return 1;
    }
    double k3 = th[SLOT_K3];
    if (model == ORA_M_2TCM_IRR) {
        /* k4 = 0: poles 0 and k2 + k3; amplitudes K1 k3/(k2+k3) (= Ki) and K1 k2/(k2+k3). */
        double beta = k2 + k3;
        rate[0] = 0.0;
        amp[0] = K1 * k3 / beta;
        rate[1] = beta;
        amp[1] = K1 * k2 / beta;
        return 2;
    }
    if (model == ORA_M_2TCM_REV) {
        double k4 = th[SLOT_K4];
        double s = k2 + k3 + k4;
        double r = sqrt(s * s - 4.0 * k2 * k4);
        double a2 = 0.5 * (s + r);
        double a1 = (2.0 * k2 * k4) / (s + r); /* = (s - r)/2 without cancellation */
        rate[0] = a1;
        amp[0] = K1 * (k3 + k4 - a1) / (a2 - a1);
        rate[1] = a2;
        amp[1] = K1 * (a2 - k3 - k4) / (a2 - a1);
        return 2;
    }
    return 0;
}

/* Gamma-variate activation of lp-ntPET (R12): 0 up to tD, peak 1 at tP. */
double ora_gamma_variate(double t, double tD, double tP, double alpha) {
    if (!(t > tD)) return 0.0;
    double s = (t - tD) / (tP - tD);
    return pow(s, alpha) * exp(alpha * (1.0 - s));
}

/* Reference-tissue models (R12): node TAC from the reference TAC cr[0..K]. */
static void simulate_reference(uint32_t model, const double* th, const double* cr, int K, double h,
                               double* out) {
    double R1 = th[SLOT_R1], k2 = th[SLOT_RK2], k2a = th[SLOT_K2A];
    if (model == ORA_M_MRTM) {
        /* C_t = R1 C_r + (k2 - R1 k2a) (exp(-k2a t) * C_r) */
        double* I = (double*)malloc(sizeof(double) * (size_t)(K + 1));
        ora_convolve_exp(k2a, cr, K, h, I);
        for (int k = 0; k <= K; ++k) out[k] = R1 * cr[k] + (k2 - R1 * k2a) * I[k];
        free(I);
        return;
    }
    /* lp-ntPET: z' = (k2 - R1 kappa) C_r - kappa z, kappa frozen at the midpoint */
    double gam = th[SLOT_GAMMA], tD = th[SLOT_TD], tP = th[SLOT_TP], alpha = th[SLOT_ALPHA];
    double z = 0.0;
    out[0] = R1 * cr[0];
    for (int k = 0; k < K; ++k) {
        double tm = ((double)k + 0.5) * h;
        double kappa = k2a + gam * ora_gamma_variate(tm, tD, tP, alpha);
        double e, a, b;
        ora_step_coeffs(kappa, h, &e, &a, &b);
        z = e * z + (k2 - R1 * kappa) * (a * cr[k] + b * cr[k + 1]);
        out[k + 1] = R1 * cr[k + 1] + z;
    }
}

/* Node TAC (Eq. (2) with C_wb = C_p for FDG):
 * C_T(t_k) = (1 - vB) sum_j A_j I_j(t_k) + vB C_p(t_k),  k = 0..K.
 * For the reference-tissue models cp is the reference TAC (R12). */
void ora_simulate_nodes(uint32_t model, const double* th, const double* cp, int K, double h,
                        double* out) {
    if (model == ORA_M_MRTM || model == ORA_M_LPNT) {
        simulate_reference(model, th, cp, K, h, out);
        return;
    }
    double rate[2], amp[2];
    int nt = ora_exp_terms(model, th, rate, amp);
    double vB = th[SLOT_VB];
    double* I = (double*)malloc(sizeof(double) * (size_t)(K + 1));
    for (int k = 0; k <= K; ++k) out[k] = 0.0;
    for (int j = 0; j < nt; ++j) {
        ora_convolve_exp(rate[j], cp, K, h, I);
        for (int k = 0; k <= K; ++k) out[k] += amp[j] * I[k];
    }
    for (int k = 0; k <= K; ++k) out[k] = (1.0 - vB) * out[k] + vB * cp[k];
    free(I);
}

/* Frame value = trapezoid of node values over the frame's nodes divided by
 * the frame length (reading R2).  kf[F+1] are the node indices of the frame
 * bounds. */
void ora_frame_average(const double* nodes, const int32_t* kf, int F, double* out) {
    for (int f = 0; f < F; ++f) {
        int a = kf[f], b = kf[f + 1];
        double s = 0.5 * nodes[a] + 0.5 * nodes[b];
        for (int k = a + 1; k < b; ++k) s += nodes[k];
        out[f] = s / (double)(b - a);
    }
}

/* Frame-averaged TACs of n parameter rows theta[n][8] (fp32, as drawn). */
void ora_simulate(uint32_t model, const float* theta, int64_t n, const double* cp, int K, double h,
                  const int32_t* kf, int F, double* out) {
    /* rows are independent; each thread works on its own rows (the result does
     * not depend on the thread count) */
#pragma omp parallel
    {
        double* nodes = (double*)malloc(sizeof(double) * (size_t)(K + 1));
        double th[ORA_NSLOT];
#pragma omp for schedule(static)
        for (int64_t r = 0; r < n; ++r) {
            for (int s = 0; s < ORA_NSLOT; ++s) th[s] = (double)theta[8 * r + s];
            ora_simulate_nodes(model, th, cp, K, h, nodes);
            ora_frame_average(nodes, kf, F, out + (size_t)F * r);
        }
        free(nodes);
    }
}

/* Same on an FP64 parameter array (used by closed-form and grid tests). */
void ora_simulate_f64(uint32_t model, const double* theta, int64_t n, const double* cp, int K,
                      double h, const int32_t* kf, int F, double* out) {
    double* nodes = (double*)malloc(sizeof(double) * (size_t)(K + 1));
    for (int64_t r = 0; r < n; ++r) {
        ora_simulate_nodes(model, theta + 8 * r, cp, K, h, nodes);
        ora_frame_average(nodes, kf, F, out + (size_t)F * r);
    }
    free(nodes);
}

/* ------------------------------------------------------------------------- */
/* Discrepancy weights and distance.                                          */
/* Sec. III-A1: sigma_t^2 is proportional to C_t exp(lambda t) / dt.  The     */
/* weight is its inverse with the (unknown) C replaced by the observed y,     */
/* floored at floor * max y (reading R3).                                     */
/* ------------------------------------------------------------------------- */
void ora_weights(const float* y, const int32_t* kf, int F, double h, double lambda, double floor_frac,
                 double* w) {
    double ymax = -INFINITY;
    for (int f = 0; f < F; ++f)
        if ((double)y[f] > ymax) ymax = (double)y[f];
    for (int f = 0; f < F; ++f) {
        double dt = (double)(kf[f + 1] - kf[f]) * h;
        double tmid = 0.5 * (double)(kf[f] + kf[f + 1]) * h;
        double yy = (double)y[f];
        double den = yy > floor_frac * ymax ? yy : floor_frac * ymax;
        w[f] = dt * exp(-lambda * tmid) / den;
    }
}

/* Reading R10: a voxel takes part only if every y_f is finite, some y_f > 0
 * and, when the caller supplies weights (wv != NULL), every weight is finite
 * and >= 0. */
static int voxel_valid(const float* y, const float* wv, int F) {
    double ymax = -INFINITY;
    for (int f = 0; f < F; ++f) {
        if (!isfinite(y[f])) return 0;
        if ((double)y[f] > ymax) ymax = (double)y[f];
        if (wv && !(isfinite(wv[f]) && wv[f] >= 0.0f)) return 0;
    }
    return ymax > 0.0;
}

/* Alg. 1 line 4 with reading R4. */
static double distance(const float* y, const double* x, const double* w, int F, int l1) {
    double d = 0.0;
    for (int f = 0; f < F; ++f) {
        double r = (double)y[f] - x[f];
        if (l1)
            d += sqrt(w[f]) * fabs(r);
        else
            d += w[f] * r * r;
    }
    return d;
}

/* ------------------------------------------------------------------------- */
/* Fixed-budget rejection ABC for every voxel (Alg. 1, Biau et al.).          */
/* ------------------------------------------------------------------------- */
typedef struct {
    double d;
    uint32_t g;
} ora_cand;

static int cand_cmp(const void* pa, const void* pb) {
    const ora_cand* a = (const ora_cand*)pa;
    const ora_cand* b = (const ora_cand*)pb;
    if (a->d < b->d) return -1;
    if (a->d > b->d) return 1;
    return (a->g < b->g) ? -1 : (a->g > b->g);
}

/* Posterior summaries of the accepted draws cand[0..n) (Eq. (6): model
 * probability = share of accepted draws; Sec. II-D3: posterior mean; Ki per
 * accepted sample, Sec. III-B2).  theta_tab, if not NULL, holds the fp32
 * parameters of every global draw index ([n_tot][8], the shared-bank form);
 * otherwise each accepted draw is regenerated from its Philox counter
 * (voxel vg, stream). */
static void summarize(const ora_cand* cand, int64_t n, int M, const uint32_t* models, const double* boxes,
                      int64_t n_draws, uint64_t seed, uint64_t vg, uint32_t stream, const float* theta_tab,
                      double* mom, double* pr) {
    float thf[8];
    for (int m = 0; m < M; ++m) {
        int slots[8];
        int np = model_params(models[m], slots);
        int use[8] = {0};
        for (int j = 0; j < np; ++j) use[slots[j]] = 1;
        const int reference = models[m] == ORA_M_MRTM || models[m] == ORA_M_LPNT;
        if (reference)
            use[SLOT_BP] = 1; /* BP_ND = k2 / k2a - 1 (Sec. II-A2) */
        else if (models[m] != ORA_M_1TCM)
            use[SLOT_KI] = 1;
        double sum[8] = {0}, sq[8] = {0};
        int64_t cnt = 0;
        for (int pass = 0; pass < 2; ++pass) {
            for (int64_t j = 0; j < n; ++j) {
                int64_t g = cand[j].g;
                if (g / n_draws != m) continue;
                int64_t i = g % n_draws;
                if (theta_tab)
                    memcpy(thf, theta_tab + 8 * g, sizeof thf);
                else
                    ora_draw(models[m], boxes + (size_t)m * 16, seed, vg, (uint64_t)i, (uint32_t)m, stream, thf,
                             NULL, NULL);
                double val[8];
                for (int s = 0; s < 8; ++s) val[s] = (double)thf[s];
                if (reference) {
                    val[SLOT_BP] = val[SLOT_RK2] / val[SLOT_K2A] - 1.0;
                } else if (use[SLOT_KI]) {
                    double K1 = val[SLOT_K1], k2 = val[SLOT_K2], k3 = val[SLOT_K3];
                    val[SLOT_KI] = K1 * k3 / (k2 + k3);
                }
                if (pass == 0) {
                    ++cnt;
                    for (int s = 0; s < 8; ++s)
                        if (use[s]) sum[s] += val[s];
                } else {
                    for (int s = 0; s < 8; ++s)
                        if (use[s]) {
                            double dv = val[s] - sum[s];
                            sq[s] += dv * dv;
                        }
                }
            }
            if (pass == 0 && cnt > 0)
                for (int s = 0; s < 8; ++s) sum[s] /= (double)cnt;
        }
        pr[m] = (double)cnt / (double)n;
        for (int s = 0; s < 8; ++s) {
            double mean = NAN, var = NAN;
            if (use[s] && cnt > 0) {
                mean = sum[s];
                var = (cnt > 1) ? sq[s] / (double)(cnt - 1) : 0.0;
            }
            mom[(size_t)m * 16 + 2 * s] = mean;
            mom[(size_t)m * 16 + 2 * s + 1] = var;
        }
    }
}

/* n = floor(N_tot * p) (remark after Alg. 1) with a 1e-6 guard against the
 * product landing just below an integer. Returns 0 if invalid. */
int64_t ora_accept_count(int64_t n_tot, double p) {
    if (!(p > 0.0 && p <= 1.0) || n_tot < 1) return 0;
    double v = floor((double)n_tot * p + 1e-6);
    int64_t n = (int64_t)v;
    if (n < 1 || n > n_tot) return 0;
    return n;
}

/*
 * y[V][F] observed TACs (fp32); cp[K+1] input at nodes (fp32 values promoted);
 * kf[F+1] frame node indices; models[M] model bits in list order;
 * boxes[M][8][2]; weights_in[V][F] optional caller weights (NULL = R3).
 * Outputs (caller-allocated):
 *   acc_g[V][n]    accepted global draw indices, ascending (d, g)
 *   acc_d[V][n]    their distances
 *   thr[V][2]      n-th and (n+1)-th smallest distance (+inf if none)
 *   moments[V][M][8][2]  mean, variance (FP64)
 *   probs[V][M]
 * Returns n, or 0 on invalid arguments.
 */
int64_t ora_infer(const float* y, int64_t V, int F, const float* cp_f32, int K, double h,
                  const int32_t* kf, const uint32_t* models, int M, const double* boxes,
                  int64_t n_draws, double p, uint64_t seed, int64_t voxel_offset, double lambda,
                  double floor_frac, int l1, const float* weights_in, int nthreads,
                  int32_t* acc_g, double* acc_d, double* thr, double* moments, double* probs) {
    int64_t n_tot = (int64_t)M * n_draws;
    int64_t n = ora_accept_count(n_tot, p);
    if (n == 0) return 0;
    double* cp = (double*)malloc(sizeof(double) * (size_t)(K + 1));
    for (int k = 0; k <= K; ++k) cp[k] = (double)cp_f32[k];
    (void)nthreads;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 1)
#endif
    for (int64_t v = 0; v < V; ++v) {
        const float* yv = y + (size_t)F * v;
        double* mom = moments + (size_t)v * M * 16;
        double* pr = probs + (size_t)v * M;
        if (!voxel_valid(yv, weights_in ? weights_in + (size_t)F * v : NULL, F)) {
            for (int j = 0; j < M * 16; ++j) mom[j] = NAN;
            for (int m = 0; m < M; ++m) pr[m] = NAN;
            for (int64_t j = 0; j < n; ++j) {
                acc_g[(size_t)v * n + j] = -1;
                acc_d[(size_t)v * n + j] = NAN;
            }
            thr[2 * v] = NAN;
            thr[2 * v + 1] = NAN;
            continue;
        }
        double* w = (double*)malloc(sizeof(double) * (size_t)F);
        double* x = (double*)malloc(sizeof(double) * (size_t)F);
        double* nodes = (double*)malloc(sizeof(double) * (size_t)(K + 1));
        ora_cand* cand = (ora_cand*)malloc(sizeof(ora_cand) * (size_t)n_tot);
        if (weights_in) {
            for (int f = 0; f < F; ++f) w[f] = (double)weights_in[(size_t)F * v + f];
        } else {
            ora_weights(yv, kf, F, h, lambda, floor_frac, w);
        }
        uint64_t vg = (uint64_t)(v + voxel_offset);
        float thf[8];
        double th[8];
        /* Alg. 1 lines 1-4: per model, n_draws prior draws, simulate, distance. */
        for (int m = 0; m < M; ++m) {
            for (int64_t i = 0; i < n_draws; ++i) {
                ora_draw(models[m], boxes + (size_t)m * 16, seed, vg, (uint64_t)i, (uint32_t)m, 0u,
                         thf, NULL, NULL);
                for (int s = 0; s < 8; ++s) th[s] = (double)thf[s];
                ora_simulate_nodes(models[m], th, cp, K, h, nodes);
                ora_frame_average(nodes, kf, F, x);
                double d = distance(yv, x, w, F, l1);
                if (isnan(d)) d = INFINITY;
                int64_t g = (int64_t)m * n_draws + i;
                cand[g].d = d;
                cand[g].g = (uint32_t)g;
            }
        }
        /* Alg. 1 line 5: the n closest, ties by lower index. */
        qsort(cand, (size_t)n_tot, sizeof(ora_cand), cand_cmp);
        for (int64_t j = 0; j < n; ++j) {
            acc_g[(size_t)v * n + j] = (int32_t)cand[j].g;
            acc_d[(size_t)v * n + j] = cand[j].d;
        }
        thr[2 * v] = cand[n - 1].d;
        thr[2 * v + 1] = (n < n_tot) ? cand[n].d : INFINITY;

        summarize(cand, n, M, models, boxes, n_draws, seed, vg, 0u, NULL, mom, pr);
        free(cand);
        free(nodes);
        free(x);
        free(w);
    }
    free(cp);
    return n;
}

/* Distances of every draw of one voxel (for parity checks near the
 * threshold): d[M * n_draws] in global draw order. */
void ora_voxel_distances(const float* yv, int F, const float* cp_f32, int K, double h,
                         const int32_t* kf, const uint32_t* models, int M, const double* boxes,
                         int64_t n_draws, uint64_t seed, int64_t v_global, double lambda,
                         double floor_frac, int l1, const float* wv, double* d_out) {
    double* cp = (double*)malloc(sizeof(double) * (size_t)(K + 1));
    for (int k = 0; k <= K; ++k) cp[k] = (double)cp_f32[k];
    double* w = (double*)malloc(sizeof(double) * (size_t)F);
    double* x = (double*)malloc(sizeof(double) * (size_t)F);
    double* nodes = (double*)malloc(sizeof(double) * (size_t)(K + 1));
    if (wv) {
        for (int f = 0; f < F; ++f) w[f] = (double)wv[f];
    } else {
        ora_weights(yv, kf, F, h, lambda, floor_frac, w);
    }
    float thf[8];
    double th[8];
    for (int m = 0; m < M; ++m)
        for (int64_t i = 0; i < n_draws; ++i) {
            ora_draw(models[m], boxes + (size_t)m * 16, seed, (uint64_t)v_global, (uint64_t)i,
                     (uint32_t)m, 0u, thf, NULL, NULL);
            for (int s = 0; s < 8; ++s) th[s] = (double)thf[s];
            ora_simulate_nodes(models[m], th, cp, K, h, nodes);
            ora_frame_average(nodes, kf, F, x);
            double d = distance(yv, x, w, F, l1);
            d_out[(size_t)m * n_draws + i] = isnan(d) ? INFINITY : d;
        }
    free(nodes);
    free(x);
    free(w);
    free(cp);
}

/* ------------------------------------------------------------------------- */
/* Shared-bank form (Alg. 1 as printed): one set of N_tot prior draws and     */
/* their simulated curves serves every voxel (Alg. 1, lines 1-3 are done      */
/* once; line 4 is a voxels x draws matrix; line 5 selects per voxel).        */
/* Bank draw i of list position m uses the Philox counter (i, 0, 1, m<<16|blk)*/
/* (stream 1; no voxel index).                                               */
/* ------------------------------------------------------------------------- */
void ora_bank(const uint32_t* models, int M, const double* boxes, int64_t n_draws, uint64_t seed,
              const float* cp_f32, int K, double h, const int32_t* kf, int F, float* theta_out, double* x_out) {
    double* cp = (double*)malloc(sizeof(double) * (size_t)(K + 1));
    for (int k = 0; k <= K; ++k) cp[k] = (double)cp_f32[k];
    const int64_t n_tot = (int64_t)M * n_draws;
    /* rows are independent; each thread works on its own rows */
#pragma omp parallel
    {
        double* nodes = (double*)malloc(sizeof(double) * (size_t)(K + 1));
#pragma omp for schedule(static)
        for (int64_t g = 0; g < n_tot; ++g) {
            const int m = (int)(g / n_draws);
            const int64_t i = g % n_draws;
            float* thf = theta_out + 8 * g;
            double th[8];
            ora_draw(models[m], boxes + (size_t)m * 16, seed, 0u, (uint64_t)i, (uint32_t)m, 1u, thf, NULL, NULL);
            for (int s = 0; s < 8; ++s) th[s] = (double)thf[s];
            ora_simulate_nodes(models[m], th, cp, K, h, nodes);
            ora_frame_average(nodes, kf, F, x_out + (size_t)F * g);
        }
        free(nodes);
    }
    free(cp);
}

int64_t ora_infer_bank(const float* y, int64_t V, int F, const float* cp_f32, int K, double h,
                       const int32_t* kf, const uint32_t* models, int M, const double* boxes, int64_t n_draws,
                       double p, uint64_t seed, double lambda, double floor_frac, int l1,
                       const float* weights_in, int nthreads, int32_t* acc_g, double* acc_d, double* thr,
                       double* moments, double* probs) {
    int64_t n_tot = (int64_t)M * n_draws;
    int64_t n = ora_accept_count(n_tot, p);
    if (n == 0) return 0;
    float* theta = (float*)malloc(sizeof(float) * 8 * (size_t)n_tot);
    double* xb = (double*)malloc(sizeof(double) * (size_t)F * (size_t)n_tot);
    ora_bank(models, M, boxes, n_draws, seed, cp_f32, K, h, kf, F, theta, xb);
    (void)nthreads;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 1)
#endif
    for (int64_t v = 0; v < V; ++v) {
        const float* yv = y + (size_t)F * v;
        double* mom = moments + (size_t)v * M * 16;
        double* pr = probs + (size_t)v * M;
        if (!voxel_valid(yv, weights_in ? weights_in + (size_t)F * v : NULL, F)) {
            for (int j = 0; j < M * 16; ++j) mom[j] = NAN;
            for (int m = 0; m < M; ++m) pr[m] = NAN;
            for (int64_t j = 0; j < n; ++j) {
                acc_g[(size_t)v * n + j] = -1;
                acc_d[(size_t)v * n + j] = NAN;
            }
            thr[2 * v] = NAN;
            thr[2 * v + 1] = NAN;
            continue;
        }
        double* w = (double*)malloc(sizeof(double) * (size_t)F);
        ora_cand* cand = (ora_cand*)malloc(sizeof(ora_cand) * (size_t)n_tot);
        if (weights_in) {
            for (int f = 0; f < F; ++f) w[f] = (double)weights_in[(size_t)F * v + f];
        } else {
            ora_weights(yv, kf, F, h, lambda, floor_frac, w);
        }
        for (int64_t g = 0; g < n_tot; ++g) {
            double d = distance(yv, xb + (size_t)F * g, w, F, l1);
            cand[g].d = isnan(d) ? INFINITY : d;
            cand[g].g = (uint32_t)g;
        }
        qsort(cand, (size_t)n_tot, sizeof(ora_cand), cand_cmp);
        for (int64_t j = 0; j < n; ++j) {
            acc_g[(size_t)v * n + j] = (int32_t)cand[j].g;
            acc_d[(size_t)v * n + j] = cand[j].d;
        }
        thr[2 * v] = cand[n - 1].d;
        thr[2 * v + 1] = (n < n_tot) ? cand[n].d : INFINITY;
        summarize(cand, n, M, models, boxes, n_draws, seed, 0u, 1u, theta, mom, pr);
        free(cand);
        free(w);
    }
    free(xb);
    free(theta);
    return n;
}

/* Posterior summaries (the reduction above: Eq. (6), Sec. II-D3, Sec. III-B2)
 * of an explicit accepted set idx[0..n) of global draw indices, for parity
 * checks of voxels whose accepted set differs from the oracle's by draws at
 * the threshold.  theta_tab != NULL: the shared-bank form (parameters of
 * every bank row); otherwise each draw is regenerated from its Philox
 * counter for voxel vg and the given stream. */
void ora_summarize_set(const int32_t* idx, int64_t n, const uint32_t* models, int M, const double* boxes,
                       int64_t n_draws, uint64_t seed, uint64_t vg, uint32_t stream, const float* theta_tab,
                       double* mom, double* pr) {
    ora_cand* cand = (ora_cand*)malloc(sizeof(ora_cand) * (size_t)(n > 0 ? n : 1));
    for (int64_t j = 0; j < n; ++j) {
        cand[j].d = 0.0;
        cand[j].g = (uint32_t)idx[j];
    }
    summarize(cand, n, M, models, boxes, n_draws, seed, vg, stream, theta_tab, mom, pr);
    free(cand);
}
