// vpet_abc.hip -- gfx950 (CDNA4) kernels and C ABI for voxelwise ABC rejection
// (vPET-ABC, arXiv 2603.14859).  The ABI is declared in include/vpet_abc.h.
//
// Design (one voxel per wavefront group, draws streamed through registers):
//  * Prior draws: Philox4x32-10 (Salmon et al., SC'11) per (voxel, draw), in
//    VGPRs; nothing about a draw is ever stored in memory (Alg. 1, lines 1-2).
//  * Forward model (Eq. (1)-(2), Alg. 1 line 3): each compartment-model
//    response is a sum of at most two decaying exponentials plus, for the
//    irreversible 2TCM, a rate-0 term.  For the piecewise-linear input, one
//    grid step of exp(-beta t) convolved with the input is exactly
//        I_{k+1} = z I_k + a C_k + b C_{k+1},  z = exp(-beta h).
//    With I_k = g H_k + b C_k and g = z b + a this becomes ONE fused
//    multiply-add per step,  H_{k+1} = z H_k + C_k,  whose C_k is the same for
//    every lane and is read through the scalar cache.  The recursion runs in
//    FP64: gfx950 issues v_fma_f64 at the rate of non-packed v_fma_f32, so the
//    accuracy costs nothing in throughput.
//  * Frame averages: the trapezoid sum of H over a frame follows from the
//    recursion itself, sum_{k=a}^{b-1} H_k = (H_a - H_b + sum C_k) / (1 - z),
//    so no per-step accumulation is needed; when 1 - z is tiny for some lane of
//    a wavefront (a nearly-zero rate) that wavefront accumulates per step
//    instead (a wave-uniform choice).
//  * Distance (Alg. 1 line 4): weighted L2 (or L1) against the observed TAC,
//    whose scaled values and weights sit in LDS and are read once per frame.
//  * Selection (Alg. 1 line 5): each wavefront keeps its voxel's running n
//    smallest 64-bit keys (fp32 distance bits << 32 | global draw index) in
//    LDS; a draw is appended only if it beats the running n-th key, and the
//    buffer is merged by a wavefront bitonic sort when full.
//  * Survivors (Eq. (6), Sec. II-D3, Sec. III-B2): the accepted draws are
//    regenerated from Philox and reduced in FP64 to per-model counts, means
//    and variances (two passes) and Ki = K1 k3 / (k2 + k3).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdarg>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <functional>
#include <condition_variable>
#include <mutex>
#include <type_traits>
#include <string>
#include <thread>
#include <vector>

#include <fcntl.h>
#include <sys/stat.h>
#include <unistd.h>

#include "vpet_abc.h"

#define VPET_VERSION_NUMBER 10000

namespace {

// Scalar-cache pointers: uniform loads through these become s_load.
typedef const __attribute__((address_space(4))) double* cdp;
typedef const __attribute__((address_space(4))) int* cip;

constexpr int kWave = 64;
// Draws per lane per tile (independent FMA chains): 4 for the one-exponential
// models, 2 where two exponentials double the per-draw state.
#ifndef VPET_DRAWS_PER_LANE
#define VPET_DRAWS_PER_LANE 4
#endif
#ifndef VPET_STEP_UNROLL
#define VPET_STEP_UNROLL 4
#endif
constexpr int kUmax = VPET_DRAWS_PER_LANE;
template <int KINDS>
constexpr int draws_per_lane() { return (KINDS == 1 || KINDS == 2) ? kUmax : 2; }
constexpr double kCmin = 1e-5;        // 1 - z below which frame sums are accumulated
constexpr int kMaxModels = 3;
constexpr int kMaxWpv = 4;
constexpr int kRedStride = 16;  // doubles per wavefront in a block reduction's scratch
constexpr uint64_t kNoKey = ~0ull;
constexpr int kLdsLimit = 65536;

enum ModelKind { KIND_1TCM = 1, KIND_IRR = 2, KIND_REV = 4, KIND_MRTM = 8, KIND_LPNT = 16 };
constexpr int kMaxParams = 7;  // lp-ntPET: R1, k2, k2a, gamma, tD, tP, alpha

// Prior box of one model in its draw order.  rel_tp (lp-ntPET): parameter 5
// (tP) is drawn in [tD + lo[5], wid[5]], i.e. lo[5] is an offset after the
// drawn tD and wid[5] holds the absolute upper bound.
struct ModelDev {
    int kind;
    int np;
    int rel_tp;
    int slot[kMaxParams];
    float lo[kMaxParams];
    float wid[kMaxParams];
};

struct Tab {
    const double* C;   // C_k, k = 0 .. kend (input at the grid nodes up to the last frame's end)
    const double* fr;  // per frame: SS (trapezoid sum of the running integral Q),
                       // PP (trapezoid sum of C), R (sum of C over the frame's steps), omega
    const int* nf;     // steps per frame
};

struct InferArgs {
    const float* tacs;
    const float* weights;
    Tab tab;
    double C0, h, floor_frac;
    int F, k0, M, cap, wpv, l1;
    long long V;
    unsigned long long vbase;
    unsigned n_draws, n_acc, key0, key1;
    ModelDev md[kMaxModels];
    float* out_mom;
    float* out_prob;
    int* out_idx;
    float* out_dist;
    float* out_thr;
    // importance-weighted ABC with a learned proposal (irreversible 2TCM only)
    const float* prop;  // [V][96] network outputs, or nullptr for prior draws
    float* out_ess;     // [V] effective sample size of the accepted weights
    float plo[4], phi[4];  // prior box of K1, k2, k3, vB (fp32)
    double prop_share;     // defensive prior share a of the proposal a p + (1 - a) q
    double prop_logscale;  // log of the sd scale of every mixture component
    double prop_logvol;    // sum_j log(phi_j - plo_j): minus the log prior density
    const float* below;    // [V] given ABC thresholds (kept draws above them do not count), or nullptr
};

// ---------------------------------------------------------------------------
// Philox4x32-10.
// ---------------------------------------------------------------------------
// a ^ b ^ c as one three-input bitwise operation (truth table 0x96, the XOR
// of the operand patterns 0xF0, 0xCC and 0xAA); the compiler emits two XORs
// when one operand is wave-uniform, as the Philox key is.
__device__ __forceinline__ uint32_t xor3(uint32_t a, uint32_t b, uint32_t c) {
    return __builtin_amdgcn_bitop3_b32(a, b, c, 0x96);
}

__device__ __forceinline__ void philox10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                         uint32_t k0, uint32_t k1, uint32_t out[4]) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t p0 = (uint64_t)0xD2511F53u * c0;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
        const uint32_t n0 = xor3((uint32_t)(p1 >> 32), c1, k0);
        const uint32_t n2 = xor3((uint32_t)(p0 >> 32), c3, k1);
        c1 = (uint32_t)p1;
        c3 = (uint32_t)p0;
        c0 = n0;
        c2 = n2;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    out[0] = c0;
    out[1] = c1;
    out[2] = c2;
    out[3] = c3;
}

__device__ __forceinline__ float unit24(uint32_t w) { return (float)(w >> 8) * 0x1p-24f; }

// Parameters of draw i of list position m for voxel v, in the model's order.
__device__ __forceinline__ void draw_params(const ModelDev& md, uint32_t key0, uint32_t key1,
                                            uint32_t v, uint32_t i, uint32_t m, float th[kMaxParams],
                                            uint32_t* words = nullptr, uint32_t stream = 0u) {
    uint32_t w[8];
    philox10(i, v, stream, m << 16, key0, key1, w);
    if (md.np > 4) {
        philox10(i, v, stream, (m << 16) | 1u, key0, key1, w + 4);
    } else {
        w[4] = w[5] = w[6] = w[7] = 0u;
    }
#pragma unroll
    for (int j = 0; j < kMaxParams; ++j) {
        float lo = md.lo[j], wid = md.wid[j];
        if (j == 5 && md.rel_tp) {  // tP in [tD + offset, hi]
            lo = th[4] + md.lo[5];
            wid = md.wid[5] - lo;
        }
        th[j] = (j < md.np) ? __builtin_fmaf(wid, unit24(w[j]), lo) : 0.0f;
    }
    if (words) {
#pragma unroll
        for (int j = 0; j < 8; ++j) words[j] = (j < 4 * ((md.np + 3) / 4)) ? w[j] : 0u;
    }
}

// ---------------------------------------------------------------------------
// Per-draw coefficients.
// ---------------------------------------------------------------------------
struct Exp1 {
    double z, H0, c, rc, eT;  // eT = (1 - vB) A g (coefficient of the trapezoid sum of H)
    double rbeta;             // 1 / beta
};

// One decaying exponential exp(-beta t), amplitude A (already times 1 - vB),
// or A = amp / beta with DIV.  Returns the b coefficient (times A) through *bA
// for the PP term.  One reciprocal serves 1/x, 1/c and 1/beta: r = 1/(x c),
// 1/x = c r, 1/c = x r, 1/beta = h/x (x = beta h > 0 here; x = 0 gives NaN
// reciprocals, which the guards below and the accumulating frame path never
// use).
// b/h = (x - (1 - e^{-x})) / x^2 = sum_{n>=0} (-x)^n / (n+2)! for 0 <= x <= 0.3,
// to n = 12 (the first omitted term is below 3e-19 of the sum).  Then
// c/x = 1 - x (b/h) and c = 1 - e^{-x} = x (c/x), neither with cancellation.
__device__ __forceinline__ double b_over_h_small(double x) {
    double p = 1.0 / 87178291200.0;  // 1/14!
    p = fma(p, -x, 1.0 / 6227020800.0);
    p = fma(p, -x, 1.0 / 479001600.0);
    p = fma(p, -x, 1.0 / 39916800.0);
    p = fma(p, -x, 1.0 / 3628800.0);
    p = fma(p, -x, 1.0 / 362880.0);
    p = fma(p, -x, 1.0 / 40320.0);
    p = fma(p, -x, 1.0 / 5040.0);
    p = fma(p, -x, 1.0 / 720.0);
    p = fma(p, -x, 1.0 / 120.0);
    p = fma(p, -x, 1.0 / 24.0);
    p = fma(p, -x, 1.0 / 6.0);
    return fma(p, -x, 0.5);
}

// c = 1 - e^{-x}, b/h and c/x for any x >= 0, out of line: it is rare on the
// usual grids, and inlined it would cost registers on every path.  b/h is
// (x - c)/x^2, or its Taylor series below x = 0.01 (cancellation).
struct ExpTerms {
    double c, bh, cx;
};
__device__ __attribute__((noinline)) ExpTerms exp_terms_general(double x) {
    ExpTerms t;
    t.c = -expm1(-x);
    const double rx = 1.0 / x;
    const double bs = 0.5 + x * (-1.0 / 6.0 + x * (1.0 / 24.0 + x * (-1.0 / 120.0 + x * (1.0 / 720.0))));
    const double bd = (x - t.c) * rx * rx;
    t.bh = (x < 0.01) ? bs : bd;
    t.cx = (x > 0.0) ? t.c * rx : 1.0;
    return t;
}

template <bool DIV = false>
__device__ __forceinline__ Exp1 exp_setup(double beta, double amp, double h, double C0, double* bA) {
    const double x = beta * h;
    // the series when every lane of the wavefront has a small step exponent
    // (a wave-uniform choice), the library expm1 otherwise
    double c, bh, cx;  // 1 - e^{-x}, b/h, c/x
    if (__ballot(!(x >= 0.0 && x <= 0.3)) == 0ull) {
        bh = b_over_h_small(x);
        cx = fma(-x, bh, 1.0);
        c = x * cx;
    } else {
        const ExpTerms t = exp_terms_general(x);
        c = t.c;
        bh = t.bh;
        cx = t.cx;
    }
    // r = 1/(x c): the hardware reciprocal estimate refined by two Newton-Raphson
    // steps, each squaring the relative error (within about an ulp of the
    // quotient; x c = 0 gives NaN, which the guards here never use)
    const double xcp = x * c;
    double r = __builtin_amdgcn_rcp(xcp);
    r = fma(r, fma(-xcp, r, 1.0), r);
    r = fma(r, fma(-xcp, r, 1.0), r);
    const double rx = c * r;
    const double rc = x * r;
    const double xc = (x > 0.0) ? x * rc : 1.0;  // x / c
    Exp1 e;
    e.rbeta = h * rx;
    if (DIV) amp *= e.rbeta;
    e.z = 1.0 - c;
    e.c = c;
    e.rc = rc;
    e.H0 = -bh * xc * xc * C0;  // H_0 = -(b / g) C_0, g = h (c/x)^2
    e.eT = amp * h * cx * cx;
    *bA = amp * h * bh;
    return e;
}

template <int KIND>
struct ModelTraits;
template <>
struct ModelTraits<KIND_1TCM> {
    static constexpr int NE = 1;
    static constexpr bool Q = false;
};
template <>
struct ModelTraits<KIND_IRR> {
    static constexpr int NE = 1;
    static constexpr bool Q = true;
};
template <>
struct ModelTraits<KIND_REV> {
    static constexpr int NE = 2;
    static constexpr bool Q = false;
};
template <>
struct ModelTraits<KIND_MRTM> {
    static constexpr int NE = 1;
    static constexpr bool Q = false;
};

template <int NE, int U>
struct DrawState {
    double z[NE][U], H[NE][U], c[NE][U], rc[NE][U], eT[NE][U];
    double e0[U], eP[U];
};

// th: parameters in model order.  Fills the per-draw state for column u.
template <int KIND, int NE, int U>
__device__ __forceinline__ void setup(const float* th, double h, double C0, DrawState<NE, U>& s,
                                      int u) {
    const double K1 = th[0], k2 = th[1];
    if constexpr (KIND == KIND_MRTM) {
        // Eq. (3) with gamma = 0: C_t = R1 C_r + (k2 - R1 k2a) exp(-k2a t) * C_r
        const double R1 = th[0], k2a = th[2];
        double bA;
        Exp1 e = exp_setup(k2a, k2 - R1 * k2a, h, C0, &bA);
        s.z[0][u] = e.z; s.H[0][u] = e.H0; s.c[0][u] = e.c; s.rc[0][u] = e.rc; s.eT[0][u] = e.eT;
        s.e0[u] = 0.0;
        s.eP[u] = R1 + bA;
    } else if constexpr (KIND == KIND_1TCM) {
        const double vB = th[2];
        const double w = 1.0 - vB;
        double bA;
        Exp1 e = exp_setup(k2, w * K1, h, C0, &bA);
        s.z[0][u] = e.z; s.H[0][u] = e.H0; s.c[0][u] = e.c; s.rc[0][u] = e.rc; s.eT[0][u] = e.eT;
        s.e0[u] = 0.0;
        s.eP[u] = vB + bA;
    } else if constexpr (KIND == KIND_IRR) {
        const double k3 = th[2], vB = th[3];
        const double w = 1.0 - vB;
        const double beta = k2 + k3;
        double bA;
        Exp1 e = exp_setup<true>(beta, w * K1 * k2, h, C0, &bA);
        s.z[0][u] = e.z; s.H[0][u] = e.H0; s.c[0][u] = e.c; s.rc[0][u] = e.rc; s.eT[0][u] = e.eT;
        s.e0[u] = w * K1 * k3 * e.rbeta;  // (1 - vB) Ki on the running integral of the input
        s.eP[u] = vB + bA;
    } else {
        const double k3 = th[2], k4 = th[3], vB = th[4];
        const double w = 1.0 - vB;
        const double sum = k2 + k3 + k4;
        const double r = sqrt(sum * sum - 4.0 * k2 * k4);
        const double sr = sum + r;
        const double a2 = 0.5 * sr;
        const double a1 = 2.0 * k2 * k4 / sr;
        const double rr = 1.0 / r;  // 1 / (a2 - a1)
        double b1, b2;
        Exp1 e1 = exp_setup(a1, w * K1 * (k3 + k4 - a1) * rr, h, C0, &b1);
        Exp1 e2 = exp_setup(a2, w * K1 * (a2 - k3 - k4) * rr, h, C0, &b2);
        s.z[0][u] = e1.z; s.H[0][u] = e1.H0; s.c[0][u] = e1.c; s.rc[0][u] = e1.rc; s.eT[0][u] = e1.eT;
        s.z[1][u] = e2.z; s.H[1][u] = e2.H0; s.c[1][u] = e2.c; s.rc[1][u] = e2.rc; s.eT[1][u] = e2.eT;
        s.e0[u] = 0.0;
        s.eP[u] = vB + b1 + b2;
    }
}

// ---------------------------------------------------------------------------
// The step/frame loop.  ACCj: exponential j accumulates its frame sums per
// step (else they come from the recursion identity).  The sink receives the
// frame value times the frame's step count, X_f = n_f x_f.
// ---------------------------------------------------------------------------
template <int NE, int U, bool Q, bool ACC0, bool ACC1, class Sink>
__device__ __forceinline__ void run_frames(const Tab& T, int F, int k0, DrawState<NE, U>& s, Sink& sink) {
    const cdp C = (cdp)T.C;
    const cdp FR = (cdp)T.fr;
    const cip NF = (cip)T.nf;
    // Two register sets for H: a frame's first step reads the set holding H at
    // the frame start and writes the other, so the start value survives the
    // frame without a copy; consecutive frames alternate the roles.
    double HA[NE][U], HB[NE][U], acc[NE][U], eD[NE][U], eA[NE][U], eR[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
        eR[u] = 0.0;
#pragma unroll
        for (int j = 0; j < NE; ++j) {
            const bool accj = (j == 0) ? ACC0 : ACC1;
            HA[j][u] = s.H[j][u];
            acc[j][u] = 0.0;
            if (accj) {  // T = acc - D/2
                eA[j][u] = s.eT[j][u];
                eD[j][u] = -0.5 * s.eT[j][u];
            } else {     // T = (1/c - 1/2) D + R / c
                eA[j][u] = 0.0;
                eD[j][u] = s.eT[j][u] * (s.rc[j][u] - 0.5);
                eR[u] = fma(s.eT[j][u], s.rc[j][u], eR[u]);
            }
        }
    }
#define VPET_STEP(H, cval)                                               \
    do {                                                                 \
        const double cc_ = (cval);                                       \
        _Pragma("unroll") for (int u = 0; u < U; ++u) {                  \
            _Pragma("unroll") for (int j = 0; j < NE; ++j) {             \
                const bool accj = (j == 0) ? ACC0 : ACC1;                \
                if (accj) acc[j][u] += H[j][u];                          \
                H[j][u] = fma(s.z[j][u], H[j][u], cc_);                  \
            }                                                            \
        }                                                                \
    } while (0)

    int k = 0;
    for (; k < k0; ++k) VPET_STEP(HA, C[k]);
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
        for (int j = 0; j < NE; ++j) acc[j][u] = 0.0;  // the steps before the first frame are not part of any frame sum

    // One frame: Hs holds H at the frame start and keeps it; Hd ends holding H
    // at the frame end (every frame has at least one step).
    auto frame = [&](int f, double (&Hs)[NE][U], double (&Hd)[NE][U]) {
        const int n = NF[f];
        const cdp Cp = C + k;
        {
            const double c0 = Cp[0];
#pragma unroll
            for (int u = 0; u < U; ++u)
#pragma unroll
                for (int j = 0; j < NE; ++j) {
                    const bool accj = (j == 0) ? ACC0 : ACC1;
                    if (accj) acc[j][u] += Hs[j][u];
                    Hd[j][u] = fma(s.z[j][u], Hs[j][u], c0);
                }
        }
        int q = 1;
#if VPET_STEP_UNROLL == 4
        for (; q + 4 <= n; q += 4) {
            const double c0 = Cp[q], c1 = Cp[q + 1], c2 = Cp[q + 2], c3 = Cp[q + 3];
            VPET_STEP(Hd, c0);
            VPET_STEP(Hd, c1);
            VPET_STEP(Hd, c2);
            VPET_STEP(Hd, c3);
        }
#endif
#pragma nounroll
        for (; q < n; ++q) VPET_STEP(Hd, Cp[q]);
        k += n;
        const double SS = FR[4 * f], PP = FR[4 * f + 1], R = FR[4 * f + 2];
        double X[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            double x = s.eP[u] * PP;
            if (Q) x = fma(s.e0[u], SS, x);
            x = fma(eR[u], R, x);
#pragma unroll
            for (int j = 0; j < NE; ++j) {
                const bool accj = (j == 0) ? ACC0 : ACC1;
                x = fma(eD[j][u], Hs[j][u] - Hd[j][u], x);
                if (accj) {
                    x = fma(eA[j][u], acc[j][u], x);
                    acc[j][u] = 0.0;
                }
            }
            X[u] = x;
        }
        sink(f, n, X);
        // The frame values are due here: left to itself the compiler defers
        // this epilogue past the next frame's steps, which then need a copy of
        // the start value of H (a move per draw and frame) and spill.
#pragma unroll
        for (int u = 0; u < U; ++u) asm volatile("" ::"v"(X[u]));
    };
    int f = 0;
    for (; f + 2 <= F; f += 2) {
        frame(f, HA, HB);
        frame(f + 1, HB, HA);
    }
    if (f < F) frame(f, HA, HB);
#undef VPET_STEP
}

__device__ __forceinline__ bool wave_all(bool p) { return __ballot(!p) == 0ull; }

// Choose the frame-sum path per exponential from a wave vote, then run.
template <int KIND, int U, class Sink>
__device__ __forceinline__ void simulate_draws(const Tab& T, int F, int k0, DrawState<ModelTraits<KIND>::NE, U>& s,
                                               Sink& sink) {
    constexpr int NE = ModelTraits<KIND>::NE;
    constexpr bool Q = ModelTraits<KIND>::Q;
    bool ok0 = true, ok1 = true;
#pragma unroll
    for (int u = 0; u < U; ++u) {
        ok0 = ok0 && (s.c[0][u] >= kCmin);
        if (NE > 1) ok1 = ok1 && (s.c[NE - 1][u] >= kCmin);
    }
    const bool id0 = wave_all(ok0);
    if constexpr (NE == 1) {
        if (id0)
            run_frames<NE, U, Q, false, false>(T, F, k0, s, sink);
        else
            run_frames<NE, U, Q, true, false>(T, F, k0, s, sink);
    } else {
        const bool id1 = wave_all(ok1);
        if (id0 && id1)
            run_frames<NE, U, Q, false, false>(T, F, k0, s, sink);
        else if (id1)
            run_frames<NE, U, Q, true, false>(T, F, k0, s, sink);
        else
            run_frames<NE, U, Q, true, true>(T, F, k0, s, sink);
    }
}

// ---------------------------------------------------------------------------
// lp-ntPET (Eq. (3)-(4)) as the ODE C_t' = R1 C_r' + k2 C_r - kappa(t) C_t with
// kappa = k2a + gamma g(t): with C_t = R1 C_r + z, z' = (k2 - R1 kappa) C_r -
// kappa z.  kappa is frozen at each step's midpoint and the step is integrated
// exactly for the reference TAC C_r linear between nodes:
//   z_{k+1} = e^{-x} z_k + (k2 - R1 kappa) (a C_k + b C_{k+1}),  x = kappa h,
//   a = h (1 - (1 + x) e^{-x}) / x^2,  b = h (e^{-x} - 1 + x) / x^2.
// g(t) = s^alpha e^{alpha (1 - s)}, s = (t - tD) / (tP - tD), for t > tD.  The
// frame value is the trapezoid sum of the node TAC.  One draw per lane.
// ---------------------------------------------------------------------------
struct StepW {
    double e, a, b;
};

__device__ __forceinline__ StepW step_weights(double kappa, double h) {
    const double x = kappa * h;
    const double c = -expm1(-x);  // 1 - e^{-x}
    const double rx2 = 1.0 / (x * x);
    // a/h = (c - x (1 - c)) / x^2 and b/h = (x - c) / x^2 lose digits for small
    // x: Taylor series below 0.01
    const double as = 0.5 + x * (-1.0 / 3.0 + x * (1.0 / 8.0 + x * (-1.0 / 30.0 + x * (1.0 / 144.0))));
    const double bs = 0.5 + x * (-1.0 / 6.0 + x * (1.0 / 24.0 + x * (-1.0 / 120.0 + x * (1.0 / 720.0))));
    StepW w;
    w.e = 1.0 - c;
    w.a = h * ((x < 0.01) ? as : (c - x * (1.0 - c)) * rx2);
    w.b = h * ((x < 0.01) ? bs : (x - c) * rx2);
    return w;
}

template <class Sink>
__device__ void simulate_lpnt(const float* th, const Tab& T, int F, int k0, double h, Sink& sink) {
    const double R1 = th[0], k2 = th[1], k2a = th[2], gam = th[3], tD = th[4], tP = th[5], alpha = th[6];
    const double rspan = 1.0 / (tP - tD);
    const StepW w0 = step_weights(k2a, h);  // the steps without activation
    const double src0 = k2 - R1 * k2a;
    const cdp C = (cdp)T.C;
    const cdp FR = (cdp)T.fr;
    const cip NF = (cip)T.nf;
    (void)FR;
    double z = 0.0, c_prev = C[0];
    int k = 0;
    auto step = [&]() {
        const double c_next = C[k + 1];
        const double tm = ((double)k + 0.5) * h;
        if (tm > tD) {
            const double sv = (tm - tD) * rspan;
            const double kap = k2a + gam * exp(alpha * (log(sv) + 1.0 - sv));
            const StepW w = step_weights(kap, h);
            z = fma(w.e, z, (k2 - R1 * kap) * fma(w.a, c_prev, w.b * c_next));
        } else {
            z = fma(w0.e, z, src0 * fma(w0.a, c_prev, w0.b * c_next));
        }
        c_prev = c_next;
        ++k;
        return fma(R1, c_next, z);  // node TAC at t_k
    };
    double ct = R1 * c_prev;
    while (k < k0) ct = step();
    for (int f = 0; f < F; ++f) {
        const int n = NF[f];
        double x = 0.5 * ct;
        for (int q = 0; q < n; ++q) {
            ct = step();
            x += (q + 1 < n) ? ct : 0.5 * ct;
        }
        const double X[1] = {x};
        sink(f, n, X);
    }
}

// ---------------------------------------------------------------------------
// Wavefront / block helpers.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

__device__ __forceinline__ int lane_id() { return (int)(threadIdx.x & 63u); }

__device__ __forceinline__ uint32_t mbcnt(uint64_t mask) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

// Bitonic sort of a[0..len) (len a power of two >= 2) by one wavefront.
__device__ void wave_bitonic_sort(uint64_t* a, int len) {
    const int lane = lane_id();
    for (int kk = 2; kk <= len; kk <<= 1) {
        for (int j = kk >> 1; j > 0; j >>= 1) {
            for (int p = lane; p < (len >> 1); p += kWave) {
                const int i = ((p & ~(j - 1)) << 1) | (p & (j - 1));
                const int l = i | j;
                const uint64_t x = a[i], y = a[l];
                const bool up = (i & kk) == 0;
                if ((x > y) == up) {
                    a[i] = y;
                    a[l] = x;
                }
            }
            wave_lds_sync();
        }
    }
}

// Same over the whole block (all waves), with barriers.
__device__ void block_bitonic_sort(uint64_t* a, int len) {
    for (int kk = 2; kk <= len; kk <<= 1) {
        for (int j = kk >> 1; j > 0; j >>= 1) {
            for (int p = threadIdx.x; p < (len >> 1); p += blockDim.x) {
                const int i = ((p & ~(j - 1)) << 1) | (p & (j - 1));
                const int l = i | j;
                const uint64_t x = a[i], y = a[l];
                const bool up = (i & kk) == 0;
                if ((x > y) == up) {
                    a[i] = y;
                    a[l] = x;
                }
            }
            __syncthreads();
        }
    }
}

// The block's n smallest keys after every wavefront has merged its own list
// (wave w's n best, sorted, at keys_all[w cap ..]): they are among the waves'
// first n keys, so for a small n those are gathered into wpv pow2(n)
// consecutive slots (padded with kNoKey) and only they are ordered: by rank
// (one key per thread, ties of the padding broken by slot) when they fit the
// block, else by a bitonic sort.  The result is keys_all[0, n) ascending
// either way.
__device__ void block_topn_sort(uint64_t* keys_all, int wpv, int cap, int n) {
    const int np2 = n <= 1 ? 1 : (1 << (32 - __builtin_clz((unsigned)(n - 1))));
    if (np2 >= cap || n > 4 * kWave) {
        block_bitonic_sort(keys_all, wpv * cap);
        return;
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    uint64_t r[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int j = lane + kWave * q;
        r[q] = j < n ? keys_all[(size_t)wave * cap + j] : kNoKey;
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int j = lane + kWave * q;
        if (j < np2) keys_all[(size_t)wave * np2 + j] = r[q];
    }
    __syncthreads();
    const int len = wpv * np2, t = (int)threadIdx.x;
    if (len > (int)blockDim.x) {
        block_bitonic_sort(keys_all, len);
        return;
    }
    uint64_t c = kNoKey;
    int rank = len;
    if (t < len) {  // len is even: two keys per 16-byte read, four reads in flight
        const ulonglong2* k2 = reinterpret_cast<const ulonglong2*>(keys_all);
        c = keys_all[t];
        rank = 0;
#pragma unroll 4
        for (int j = 0; j < (len >> 1); ++j) {
            const ulonglong2 o = k2[j];
            rank += (o.x < c || (o.x == c && 2 * j < t)) ? 1 : 0;
            rank += (o.y < c || (o.y == c && 2 * j + 1 < t)) ? 1 : 0;
        }
    }
    __syncthreads();
    if (rank < n) keys_all[rank] = c;
    __syncthreads();
}

// Running top-n of one wavefront: keys[0, n) is the sorted set (padded with
// kNoKey), keys[n, n + nbuf) the unsorted candidates, keys[.., cap) free.
struct TopN {
    uint64_t* keys;
    int n, cap, nbuf;
    uint64_t tau;

    // Sorts only pow2(n + nbuf) keys: the slots above hold kNoKey or keys
    // dropped by an earlier merge, none of which can re-enter the top n.
    __device__ void merge() {
        const int used = n + nbuf;
        const int len = used <= 2 ? 2 : min(cap, 1 << (32 - __builtin_clz((unsigned)(used - 1))));
        for (int j = used + lane_id(); j < len; j += kWave) keys[j] = kNoKey;
        wave_lds_sync();
        wave_bitonic_sort(keys, len);
        tau = keys[n - 1];
        nbuf = 0;
    }

    // One column of 64 keys at a time, so the buffer (cap - n >= 128 keys)
    // always has room for a column after a merge.
    template <int U>
    __device__ void insert(const uint64_t (&key)[U]) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
            uint64_t b = __ballot(key[u] < tau);
            if (b == 0ull) continue;
            if (nbuf + __popcll(b) > cap - n) {
                merge();
                b = __ballot(key[u] < tau);
            }
            if (key[u] < tau) keys[n + nbuf + (int)mbcnt(b)] = key[u];
            nbuf += __popcll(b);
            wave_lds_sync();
        }
    }
};

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
    return v;
}

// FP64 lane exchange by a DPP pattern within rows of 16 lanes (two 32-bit
// moves; no LDS round trip).
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v) {
    const uint64_t u = __builtin_bit_cast(uint64_t, v);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_mov_dpp((int)(uint32_t)u, CTRL, 0xF, 0xF, false);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_mov_dpp((int)(uint32_t)(u >> 32), CTRL, 0xF, 0xF, false);
    return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}
__device__ __forceinline__ double lane_f64(double v, int l) {
    const uint64_t u = __builtin_bit_cast(uint64_t, v);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)u, l);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(u >> 32), l);
    return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}
// FP64 wavefront sum, the same value in every lane: pairs, quads, halves and
// whole rows of 16 by DPP (each step adds the mirror lane's partial, so the
// lanes of a row agree), then (row0 + row1) + (row2 + row3).
template <>
__device__ __forceinline__ double wave_sum<double>(double v) {
    v += dpp_f64<0xB1>(v);   // quad_perm [1,0,3,2]
    v += dpp_f64<0x4E>(v);   // quad_perm [2,3,0,1]
    v += dpp_f64<0x141>(v);  // row_half_mirror
    v += dpp_f64<0x140>(v);  // row_mirror
    return (lane_f64(v, 0) + lane_f64(v, 16)) + (lane_f64(v, 32) + lane_f64(v, 48));
}
__device__ __forceinline__ double wave_max(double v) {
    v = fmax(v, dpp_f64<0xB1>(v));
    v = fmax(v, dpp_f64<0x4E>(v));
    v = fmax(v, dpp_f64<0x141>(v));
    v = fmax(v, dpp_f64<0x140>(v));
    return fmax(fmax(lane_f64(v, 0), lane_f64(v, 16)), fmax(lane_f64(v, 32), lane_f64(v, 48)));
}

// Sum of NV values over the block; every thread gets the totals.
template <int NV>
__device__ void block_sum(double (&v)[NV], double* red, int wpv) {
    static_assert(NV <= kRedStride, "reduction scratch per wavefront");
    const int wave = threadIdx.x >> 6;
#pragma unroll
    for (int q = 0; q < NV; ++q) v[q] = wave_sum(v[q]);
    if (lane_id() == 0)
#pragma unroll
        for (int q = 0; q < NV; ++q) red[wave * kRedStride + q] = v[q];
    __syncthreads();
#pragma unroll
    for (int q = 0; q < NV; ++q) {
        double t = 0.0;
        for (int w = 0; w < wpv; ++w) t += red[w * kRedStride + q];
        v[q] = t;
    }
    __syncthreads();
}

// ---------------------------------------------------------------------------
// Sinks.
// ---------------------------------------------------------------------------
// X is the frame's node sum (n_f times its average).  L2: yw[f] = (s y_f,
// s / n_f) with s = sqrt(w_f), so r = s (y - X / n_f) is one FMA and
// d += r^2 another.  L1: yw[f] = (n_f y_f, sqrt(w_f) / n_f).
template <int U, bool L1>
struct DistSink {
    const double2* yw;
    double d[U];
    __device__ __forceinline__ void operator()(int f, int, const double (&X)[U]) {
        const double2 q = yw[f];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            if (L1) {
                d[u] = fma(q.y, fabs(q.x - X[u]), d[u]);
            } else {
                const double r = fma(-q.y, X[u], q.x);
                d[u] = fma(r, r, d[u]);
            }
        }
    }
};

struct TacSink {
    float* out;  // row base, or nullptr for a padding lane
    __device__ __forceinline__ void operator()(int f, int n, const double (&X)[1]) {
        if (out) out[f] = (float)(X[0] / (double)n);
    }
};

// ---------------------------------------------------------------------------
// Kernels.
// ---------------------------------------------------------------------------
template <int KIND, int U, bool L1>
__device__ __forceinline__ void tile_keys(const InferArgs& P, int m, uint32_t v, uint32_t i0,
                                          const double2* yw, uint64_t (&key)[U]) {
    const ModelDev& md = P.md[m];
    constexpr int NE = ModelTraits<KIND>::NE;
    DrawState<NE, U> s;
    uint32_t idx[U];
    bool ok[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const uint32_t i = i0 + (uint32_t)(u * kWave + lane_id());
        ok[u] = i < P.n_draws;
        idx[u] = ok[u] ? i : P.n_draws - 1;
        float th[kMaxParams];
        draw_params(md, P.key0, P.key1, v, idx[u], (uint32_t)m, th);
        setup<KIND, NE, U>(th, P.h, P.C0, s, u);
    }
    DistSink<U, L1> sink;
    sink.yw = yw;
#pragma unroll
    for (int u = 0; u < U; ++u) sink.d[u] = 0.0;
    simulate_draws<KIND, U>(P.tab, P.F, P.k0, s, sink);
#pragma unroll
    for (int u = 0; u < U; ++u) {
        float fd = (float)sink.d[u];
        if (!(fd == fd)) fd = __builtin_inff();
        const uint32_t g = (uint32_t)m * P.n_draws + idx[u];
        key[u] = ok[u] ? (((uint64_t)__float_as_uint(fd) << 32) | g) : kNoKey;
    }
}

// Slot values (K1, k2, k3, k4, vB, Ki) of an accepted draw.
__device__ __forceinline__ void slot_values(int kind, const float th[5], double val[6]) {
    val[0] = th[0];
    val[1] = th[1];
    if (kind == KIND_1TCM) {
        val[2] = 0.0; val[3] = 0.0; val[4] = th[2]; val[5] = 0.0;
    } else if (kind == KIND_IRR) {
        val[2] = th[2]; val[3] = 0.0; val[4] = th[3];
        val[5] = val[0] * val[2] / (val[1] + val[2]);
    } else {
        val[2] = th[2]; val[3] = th[3]; val[4] = th[4];
        val[5] = val[0] * val[2] / (val[1] + val[2]);
    }
}

__device__ __forceinline__ bool slot_used(int kind, int q) {
    if (q == 5) return kind != KIND_1TCM;
    if (kind == KIND_1TCM) return q == 0 || q == 1 || q == 4;
    if (kind == KIND_IRR) return q != 3;
    return true;
}

// KINDS: the one model kind of a single-model call (a smaller kernel with
// fewer live registers), or 0 for any mix of models.
template <int KINDS, bool L1>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) void vpet_infer_kernel(InferArgs P) {
    extern __shared__ __align__(16) unsigned char lds[];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const long long row = blockIdx.x;
    if (row >= P.V) return;
    const int F = P.F;
    const uint32_t vg = (uint32_t)(P.vbase + (unsigned long long)row);
    double2* yw = reinterpret_cast<double2*>(lds);
    const int yw_bytes = (16 * F + 15) & ~15;
    uint64_t* keys_all = reinterpret_cast<uint64_t*>(lds + yw_bytes);
    double* red = reinterpret_cast<double*>(keys_all + (size_t)P.wpv * P.cap);
    int* flag = reinterpret_cast<int*>(red + kRedStride * kMaxWpv);
    const int n = (int)P.n_acc;

    // Observed curve, validity and scaled weights (wave 0).
    if (wave == 0) {
        const float* y = P.tacs + (size_t)row * F;
        const cdp FR = (cdp)P.tab.fr;
        const cip NF = (cip)P.tab.nf;
        float ymax = -__builtin_inff();
        int bad = 0;
        for (int f = lane; f < F; f += kWave) {
            const float yy = y[f];
            bad |= !isfinite(yy);
            ymax = fmaxf(ymax, yy);
            if (P.weights) {  // caller weights must be finite and >= 0
                const float wv = P.weights[(size_t)row * F + f];
                bad |= !(wv >= 0.0f) || !isfinite(wv);
            }
        }
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
            ymax = fmaxf(ymax, __shfl_xor(ymax, off, kWave));
            bad |= __shfl_xor(bad, off, kWave);
        }
        const bool valid = !bad && ymax > 0.0f;
        const double den_floor = P.floor_frac * (double)ymax;
        for (int f = lane; f < F; f += kWave) {
            const double nfd = (double)NF[f];
            const double yy = (double)y[f];
            double w;
            if (P.weights) {
                w = (double)P.weights[(size_t)row * F + f];
            } else {
                const double den = yy > den_floor ? yy : den_floor;
                w = FR[4 * f + 3] / den;
            }
            const double sw = sqrt(w);
            yw[f] = P.l1 ? make_double2(nfd * yy, sw / nfd) : make_double2(sw * yy, sw / nfd);
        }
        if (lane == 0) *flag = valid ? 1 : 0;
    }
    __syncthreads();
    if (*flag == 0) {
        if (wave == 0) {
            const float qnan = __builtin_nanf("");
            for (int j = lane; j < P.M * 16; j += kWave) P.out_mom[(size_t)row * P.M * 16 + j] = qnan;
            for (int j = lane; j < P.M; j += kWave) P.out_prob[(size_t)row * P.M + j] = qnan;
            if (P.out_idx)
                for (int j = lane; j < n; j += kWave) P.out_idx[(size_t)row * n + j] = -1;
            if (P.out_dist)
                for (int j = lane; j < n; j += kWave) P.out_dist[(size_t)row * n + j] = qnan;
            if (P.out_thr && lane == 0) P.out_thr[row] = qnan;
        }
        return;
    }

    // Stream every draw of every model through the wave's running top-n.
    TopN top;
    top.keys = keys_all + (size_t)wave * P.cap;
    top.n = n;
    top.cap = P.cap;
    top.nbuf = 0;
    top.tau = kNoKey;
    for (int j = lane; j < P.cap; j += kWave) top.keys[j] = kNoKey;
    wave_lds_sync();
    constexpr int kU = draws_per_lane<KINDS>();
    constexpr int kTile = kWave * kU;
    const uint32_t ntiles = (P.n_draws + kTile - 1) / kTile;
    for (int m = 0; m < P.M; ++m) {
        const int kind = KINDS != 0 ? KINDS : P.md[m].kind;
        for (uint32_t t = (uint32_t)wave; t < ntiles; t += (uint32_t)P.wpv) {
            uint64_t key[kU];
            if constexpr (KINDS != 0)
                tile_keys<KINDS, kU, L1>(P, m, vg, t * kTile, yw, key);
            else if (kind == KIND_IRR)
                tile_keys<KIND_IRR, kU, L1>(P, m, vg, t * kTile, yw, key);
            else if (kind == KIND_REV)
                tile_keys<KIND_REV, kU, L1>(P, m, vg, t * kTile, yw, key);
            else
                tile_keys<KIND_1TCM, kU, L1>(P, m, vg, t * kTile, yw, key);
            top.insert(key);
        }
    }
    top.merge();
    __syncthreads();
    if (P.wpv > 1) block_topn_sort(keys_all, P.wpv, P.cap, n);
    const uint64_t* acc = keys_all;  // the n accepted keys, ascending

    if (P.out_idx)
        for (int j = tid; j < n; j += blockDim.x) P.out_idx[(size_t)row * n + j] = (int)(uint32_t)acc[j];
    if (P.out_dist)
        for (int j = tid; j < n; j += blockDim.x) P.out_dist[(size_t)row * n + j] = __uint_as_float((uint32_t)(acc[j] >> 32));
    if (P.out_thr && tid == 0) P.out_thr[row] = __uint_as_float((uint32_t)(acc[n - 1] >> 32));

    // Survivor reduction per model: count, mean, variance (two passes, FP64).
    for (int m = 0; m < P.M; ++m) {
        const ModelDev& md = P.md[m];
        double s1[7];
#pragma unroll
        for (int q = 0; q < 7; ++q) s1[q] = 0.0;
        for (int j = tid; j < n; j += blockDim.x) {
            const uint32_t g = (uint32_t)acc[j];
            if (g / P.n_draws != (uint32_t)m) continue;
            float th[kMaxParams];
            draw_params(md, P.key0, P.key1, vg, g - (uint32_t)m * P.n_draws, (uint32_t)m, th);
            double val[6];
            slot_values(md.kind, th, val);
#pragma unroll
            for (int q = 0; q < 6; ++q) s1[q] += val[q];
            s1[6] += 1.0;
        }
        block_sum<7>(s1, red, P.wpv);
        const double cnt = s1[6];
        double mean[6];
#pragma unroll
        for (int q = 0; q < 6; ++q) mean[q] = s1[q] / cnt;
        double s2[6];
#pragma unroll
        for (int q = 0; q < 6; ++q) s2[q] = 0.0;
        for (int j = tid; j < n; j += blockDim.x) {
            const uint32_t g = (uint32_t)acc[j];
            if (g / P.n_draws != (uint32_t)m) continue;
            float th[kMaxParams];
            draw_params(md, P.key0, P.key1, vg, g - (uint32_t)m * P.n_draws, (uint32_t)m, th);
            double val[6];
            slot_values(md.kind, th, val);
#pragma unroll
            for (int q = 0; q < 6; ++q) {
                const double dv = val[q] - mean[q];
                s2[q] = fma(dv, dv, s2[q]);
            }
        }
        block_sum<6>(s2, red, P.wpv);
        if (tid < 16) {
            const int q = tid >> 1;
            float outv = __builtin_nanf("");
            if (q < 6 && slot_used(md.kind, q) && cnt > 0.0) {
                if ((tid & 1) == 0)
                    outv = (float)mean[q];
                else
                    outv = (cnt > 1.0) ? (float)(s2[q] / (cnt - 1.0)) : 0.0f;
            }
            P.out_mom[((size_t)row * P.M + m) * 16 + tid] = outv;
        }
        if (tid == 0) P.out_prob[(size_t)row * P.M + m] = (float)(cnt / (double)n);
    }
}

template <int KIND>
__global__ __launch_bounds__(256) void vpet_simulate_kernel(const float* __restrict__ theta, long long n, Tab T,
                                                            double C0, double h, int F, int k0, float* out) {
    const long long row = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const bool ok = row < n;
    const long long r = ok ? row : n - 1;
    float th[kMaxParams] = {};
    const float* t = theta + (size_t)r * VPET_PSTRIDE;
    if (KIND == KIND_1TCM) {
        th[0] = t[0]; th[1] = t[1]; th[2] = t[4];
    } else if (KIND == KIND_IRR) {
        th[0] = t[0]; th[1] = t[1]; th[2] = t[2]; th[3] = t[4];
    } else if (KIND == KIND_REV) {
        th[0] = t[0]; th[1] = t[1]; th[2] = t[2]; th[3] = t[3]; th[4] = t[4];
    } else {  // reference-tissue models: slots are the draw order
        for (int j = 0; j < (KIND == KIND_LPNT ? 7 : 3); ++j) th[j] = t[j];
    }
    TacSink sink{ok ? out + (size_t)row * F : nullptr};
    if constexpr (KIND == KIND_LPNT) {
        simulate_lpnt(th, T, F, k0, h, sink);
    } else {
        constexpr int NE = ModelTraits<KIND>::NE;
        DrawState<NE, 1> s;
        setup<KIND, NE, 1>(th, h, C0, s, 0);
        simulate_draws<KIND, 1>(T, F, k0, s, sink);
    }
}

__global__ __launch_bounds__(256) void vpet_draws_kernel(ModelDev md0, ModelDev md1, ModelDev md2, int M,
                                                         uint32_t key0, uint32_t key1, const int64_t* voxel,
                                                         const int64_t* draw, const int32_t* mpos, long long count,
                                                         uint32_t* out_words, float* out_theta) {
    const long long j = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= count) return;
    const int m = mpos[j];
    float* th_out = out_theta + (size_t)j * VPET_PSTRIDE;
    uint32_t* w_out = out_words + (size_t)j * 8;
    for (int q = 0; q < VPET_PSTRIDE; ++q) th_out[q] = __builtin_nanf("");
    for (int q = 0; q < 8; ++q) w_out[q] = 0u;
    if (m < 0 || m >= M) return;
    const ModelDev& md = (m == 0) ? md0 : (m == 1 ? md1 : md2);
    float th[kMaxParams];
    uint32_t words[8];
    draw_params(md, key0, key1, (uint32_t)voxel[j], (uint32_t)draw[j], (uint32_t)m, th, words);
    for (int q = 0; q < 8; ++q) w_out[q] = words[q];
    for (int q = 0; q < md.np; ++q) th_out[md.slot[q]] = th[q];
}

// ===========================================================================
// Shared-bank form (Alg. 1 as printed): one bank of draws and curves for all
// voxels.  Bank draw i of list position m uses the Philox counter
// (i, 0, 1, m << 16 | blk): stream 1, no voxel index.
// ===========================================================================
constexpr int kBankTopK = 16;  // pilot: each voxel's 16th smallest distance over a bank prefix

struct BankSink {
    double* row;  // bank row of this draw, or nullptr for a padding lane
    __device__ __forceinline__ void operator()(int f, int n, const double (&X)[1]) {
        if (row) row[f] = X[0] / (double)n;
    }
};

// One thread per bank draw of one model: parameters and frame averages.
template <int KIND>
__global__ __launch_bounds__(256) void vpet_bank_kernel(ModelDev md, int m, unsigned n_draws, unsigned key0,
                                                        unsigned key1, Tab T, double C0, double h, int F, int k0,
                                                        int ld, float* theta_out, double* x_out) {
    const unsigned i = blockIdx.x * blockDim.x + threadIdx.x;
    const bool ok = i < n_draws;
    const unsigned ii = ok ? i : n_draws - 1;
    const size_t g = (size_t)m * n_draws + ii;
    float th[kMaxParams];
    draw_params(md, key0, key1, 0u, ii, (uint32_t)m, th, nullptr, 1u);
    if (ok) {
        float* to = theta_out + g * VPET_PSTRIDE;
        for (int q = 0; q < VPET_PSTRIDE; ++q) to[q] = __builtin_nanf("");
        for (int q = 0; q < md.np; ++q) to[md.slot[q]] = th[q];
        double* row = x_out + g * (size_t)ld;
        for (int f = F; f < ld; ++f) row[f] = 0.0;  // padding frames contribute nothing
    }
    BankSink sink{ok ? x_out + g * (size_t)ld : nullptr};
    if constexpr (KIND == KIND_LPNT) {
        simulate_lpnt(th, T, F, k0, h, sink);
    } else {
        constexpr int NE = ModelTraits<KIND>::NE;
        DrawState<NE, 1> s;
        setup<KIND, NE, 1>(th, h, C0, s, 0);
        simulate_draws<KIND, 1>(T, F, k0, s, sink);
    }
}

struct BankArgs {
    const float* tacs;
    const float* weights;
    const double* omega;    // per frame: dt_f exp(-lambda tmid_f)
    const double* bank_x;   // [N][ld] frame averages (zero padding)
    const float* bank_theta;
    double floor_frac;
    int F, ld, l1, M, cap, fb_cap;
    int scap;               // keys the re-ranking select holds in LDS (a power of two)
    long long V;            // voxels in this launch
    unsigned n_tot, n_draws, n_acc, n_pilot;
    int kinds[kMaxModels];
    float* tau;             // [V] pilot threshold (fp32 distance), NaN for an invalid voxel
    int* cnt;               // [V] candidates found (may exceed cap)
    int* cnt_hi;            // [V] of them, in the second half of the list (the rest are at its start)
    uint64_t* cand;         // [V][cap] candidate keys
    int* fb_list;           // [V] voxels whose candidate list cannot certify the top n
    unsigned* fb_count;     // [1] entries in fb_list
    // BF16 contraction (L2 only): d = a_v + sum_k A_vk B_gk with
    // A_v = [-2 w y, w], B_g = [x, x^2], each split into bf16 hi + lo parts
    int K;                  // 2 * ld
    uint16_t* bhi;          // [N][K]
    uint16_t* blo;
    uint16_t* ahi;          // [V][K]
    uint16_t* alo;
    float* cthr;            // [V] candidate test: computed sum_k A B <= cthr
    float* tau1;            // [V] a tighter first threshold (contraction scan), with
    float* cthr1;           // [V] its candidate test; rows passing it are re-ranked first
    double* aval;           // [V] a_v = sum_f w y^2; NaN for an invalid voxel
    float* out_mom;
    float* out_prob;
    int* out_idx;
    float* out_dist;
    float* out_thr;
    // Grouped banks (learned proposal): the voxels of this launch are
    // positions pos0 + row of a grouped order, position p belongs to group
    // p / grp_vox and is screened against that group's grp_rows bank rows,
    // which start at row (p / grp_vox - g0) grp_rows of bank_x / bank_theta.
    // grp_vox = 0: one bank of n_tot rows for every voxel.
    long long pos0, g0;
    unsigned grp_vox, grp_rows;
    const double* bank_logw;  // [rows] log importance weight of each bank row, or nullptr (weight 1)
    const int* out_row;       // [positions] output row of each position, or nullptr (the launch row)
    float* out_ess;           // [V] effective sample size of the accepted weights (with bank_logw)
    const float* below;       // [V] given ABC thresholds (by output row), or nullptr
    // [groups of the launch][ld] FP64 reference curve of each group (grouped
    // banks), or nullptr: the BF16 screen works on y - r and x - r
    const double* ref;
};

// First bank row of the bank that voxel `row` of the launch is screened against.
__device__ __forceinline__ unsigned bank_row_base(const BankArgs& P, long long row) {
    if (P.grp_vox == 0u) return 0u;
    return (unsigned)(((unsigned long long)(P.pos0 + row) / P.grp_vox - (unsigned long long)P.g0) * P.grp_rows);
}
__device__ __forceinline__ long long bank_out_row(const BankArgs& P, long long row) {
    return P.out_row ? (long long)P.out_row[P.pos0 + row] : row;
}
// Position in a voxel's list of its j-th candidate (c0 of them at the start,
// the rest from the middle on).
__device__ __forceinline__ int cand_slot(const BankArgs& P, int j, int c0) {
    return j < c0 ? j : (P.cap >> 1) + (j - c0);
}

// Per-lane observed curve and weights of voxel `row` (a lane per voxel).
template <int LD, bool L1>
__device__ __forceinline__ bool lane_curve(const BankArgs& P, long long row, double (&Y)[LD], double (&Wt)[LD]) {
    const float* y = P.tacs + (size_t)row * P.F;
    float ymax = -__builtin_inff();
    bool bad = false;
#pragma unroll
    for (int f = 0; f < LD; ++f) {
        const float yy = (f < P.F) ? y[f] : 0.0f;
        bad = bad || !isfinite(yy);
        ymax = fmaxf(ymax, (f < P.F) ? yy : -__builtin_inff());
        Y[f] = (double)yy;
    }
    const double den_floor = P.floor_frac * (double)ymax;
    const cdp OM = (cdp)P.omega;
#pragma unroll
    for (int f = 0; f < LD; ++f) {
        double w = 0.0;
        if (f < P.F) {
            if (P.weights) {  // caller weights must be finite and >= 0
                w = (double)P.weights[(size_t)row * P.F + f];
                bad = bad || !(w >= 0.0) || !isfinite(w);
            } else {
                w = OM[f] / (Y[f] > den_floor ? Y[f] : den_floor);
            }
            if (L1) w = sqrt(w);
        }
        Wt[f] = w;
    }
    return !bad && ymax > 0.0f;
}

// Exact distance of a bank row to a voxel, in one fixed order on every path:
// four partial sums over consecutive quarters of the (padded) frames, each an
// FMA chain in frame order, added as (p0 + p1) + (p2 + p3).  The re-ranking
// select computes a quarter per lane (four lanes per row); the FP64 scan and
// the exact fallback compute all four in one lane.  A row therefore has the
// same FP64 distance whichever path ranks it.
template <bool L1>
__device__ __forceinline__ double dist_term(double y, double w, double x, double acc) {
    const double r = y - x;
    return L1 ? fma(w, fabs(r), acc) : fma(w * r, r, acc);
}

// The row is wave-uniform (FP64 scan), so its values are scalar operands.
template <int LD, bool L1>
__device__ __forceinline__ double bank_distance(cdp xr, const double (&Y)[LD], const double (&Wt)[LD]) {
    constexpr int Q = LD / 4;
    double p[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        p[t] = 0.0;
#pragma unroll
        for (int f = t * Q; f < (t + 1) * Q; ++f) p[t] = dist_term<L1>(Y[f], Wt[f], xr[f], p[t]);
    }
    return (p[0] + p[1]) + (p[2] + p[3]);
}

// The same from a per-lane row pointer (exact fallback).
template <int LD, bool L1>
__device__ __forceinline__ double row_distance(const double* xr, const double (&Y)[LD], const double (&Wt)[LD]) {
    constexpr int Q = LD / 4;
    double p[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        p[t] = 0.0;
#pragma unroll
        for (int f = t * Q; f < (t + 1) * Q; ++f) p[t] = dist_term<L1>(Y[f], Wt[f], xr[f], p[t]);
    }
    return (p[0] + p[1]) + (p[2] + p[3]);
}

// The voxel's curve and weights (as lane_curve computes them, padding frames
// 0) written once to LDS by the first LD lanes of a wavefront; every lane then
// reads them as broadcast operands.
template <int LD, bool L1>
__device__ __forceinline__ void wave_curve_lds(const BankArgs& P, long long row, float yy, double* Ys,
                                               double* Ws) {
    const int f = lane_id();  // yy: the TAC value of frame f (0 past the last frame)
    float ymax = (f < P.F) ? yy : -__builtin_inff();
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) ymax = fmaxf(ymax, __shfl_xor(ymax, off, kWave));
    const double den_floor = P.floor_frac * (double)ymax;
    double w = 0.0;
    if (f < P.F) {
        if (P.weights) {
            w = (double)P.weights[(size_t)row * P.F + f];
        } else {
            const double Y = (double)yy;
            w = P.omega[f] / (Y > den_floor ? Y : den_floor);
        }
        if (L1) w = sqrt(w);
    }
    if (f < LD) {
        Ys[f] = (double)yy;
        Ws[f] = w;
    }
    wave_lds_sync();
}

__device__ __forceinline__ float key_dist(double d) {
    float fd = (float)d;
    return (fd == fd) ? fd : __builtin_inff();
}

// PILOT: each lane's 16 smallest distances over n_pilot bank rows spread evenly
// over the bank (it is ordered by model) ->
// tau.  SCAN: every bank row; rows with fp32 distance <= tau are appended to
// the voxel's candidate list.
template <int LD, bool L1, bool PILOT>
__global__ __launch_bounds__(256) void vpet_bank_scan_kernel(BankArgs P) {
    const long long row0 = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const bool live = row0 < P.V;
    const long long row = live ? row0 : P.V - 1;
    double Y[LD], Wt[LD];
    const bool valid = lane_curve<LD, L1>(P, row, Y, Wt);
    // a block's 256 voxels share one bank (groups hold whole 256-voxel tiles)
    const unsigned gb = bank_row_base(P, (long long)blockIdx.x * blockDim.x);
    const cdp X = (cdp)(P.bank_x + (size_t)gb * LD);
    if (PILOT) {
        float top[kBankTopK];
#pragma unroll
        for (int q = 0; q < kBankTopK; ++q) top[q] = __builtin_inff();
        for (unsigned j = 0; j < P.n_pilot; ++j) {
            // pilot rows spread evenly over the bank (it is ordered by model)
            const unsigned g = (unsigned)(((uint64_t)j * P.n_tot) / P.n_pilot);
            const float fd = key_dist(bank_distance<LD, L1>(X + (size_t)g * LD, Y, Wt));
            if (fd < top[kBankTopK - 1]) {  // insert into the sorted list
#pragma unroll
                for (int q = kBankTopK - 1; q > 0; --q)
                    top[q] = (fd < top[q - 1]) ? top[q - 1] : ((fd < top[q]) ? fd : top[q]);
                top[0] = fminf(top[0], fd);
            }
        }
        if (live) P.tau[row] = valid ? top[kBankTopK - 1] : __builtin_nanf("");
    } else {
        const float tau = P.tau[row];
        uint64_t* out = P.cand + (size_t)row * P.cap;
        int c = 0;
        for (unsigned g = 0; g < P.n_tot; ++g) {
            const float fd = key_dist(bank_distance<LD, L1>(X + (size_t)g * LD, Y, Wt));
            if (fd <= tau) {
                if (c < P.cap) out[c] = ((uint64_t)__float_as_uint(fd) << 32) | (gb + g);
                ++c;
            }
        }
        if (live) {
            P.cnt[row] = valid ? c : -1;
            P.cnt_hi[row] = 0;
        }
    }
}

// Canonical slot values of a bank draw (bank_theta rows are already in slot
// order) with the derived slot: Ki = K1 k3 / (k2 + k3) for the 2TCMs, BP_ND =
// k2 / k2a - 1 for the reference-tissue models; unused slots 0.
__device__ __forceinline__ bool bank_slot_used(int kind, int q) {
    switch (kind) {
        case KIND_1TCM: return q == 0 || q == 1 || q == 4;
        case KIND_IRR: return q <= 5 && q != 3;
        case KIND_REV: return q <= 5;
        case KIND_MRTM: return q <= 2 || q == 7;
        default: return true;  // lp-ntPET: all seven parameters and BP_ND
    }
}

__device__ __forceinline__ void bank_slot_values(int kind, const float* t, double (&val)[8]) {
#pragma unroll
    for (int q = 0; q < 8; ++q) val[q] = bank_slot_used(kind, q) ? (double)t[q] : 0.0;
    if (kind == KIND_IRR || kind == KIND_REV) val[5] = val[0] * val[2] / (val[1] + val[2]);
    if (kind == KIND_MRTM || kind == KIND_LPNT) val[7] = val[1] / val[2] - 1.0;
}

__device__ double block_max(double v, double* red, int nw);
constexpr int kOutCache = 2;   // accepted keys per thread whose values the output passes keep in registers
constexpr int kOutCacheW = 1;  // the same with importance weights

// Weighted outputs (bank rows with log weights, the learned-proposal bank):
// of the n accepted keys those at or below the voxel's given threshold (if
// any) count with weight w = exp(log w - max); per model m the probability
// sum_m w / sum w and the weighted mean and variance sum w (t - mean)^2 /
// sum w of every slot; the ESS (sum w)^2 / sum w^2 over every model.
__device__ void bank_outputs_weighted(const BankArgs& P, long long row, long long orow, const uint64_t* acc,
                                      double* red) {
    const int n = (int)P.n_acc;
    const int tid = threadIdx.x, nw = blockDim.x >> 6;
    const unsigned gb = bank_row_base(P, row);
    const float h_v = P.below ? P.below[orow] : __builtin_inff();
    auto log_w = [&](int j, double& lw) {
        if (acc[j] == kNoKey || !(__uint_as_float((uint32_t)(acc[j] >> 32)) <= h_v)) return false;
        lw = P.bank_logw[(uint32_t)acc[j]];
        return lw > -__builtin_inf();
    };
    // the first kOutCacheW keys of this thread keep their log weight, weight
    // and values in registers across the passes (the same sums in the same
    // order as reading them again; one key, to stay within the registers of
    // four wavefronts per SIMD)
    double c_lw[kOutCacheW], c_w[kOutCacheW], c_val[kOutCacheW][8];
    bool c_ok[kOutCacheW];
    double lmax = -__builtin_inf();
#pragma unroll
    for (int i = 0; i < kOutCacheW; ++i) {
        const int j = tid + i * (int)blockDim.x;
        c_ok[i] = j < n && log_w(j, c_lw[i]);
        if (c_ok[i]) lmax = fmax(lmax, c_lw[i]);
    }
    for (int j = tid + kOutCacheW * (int)blockDim.x; j < n; j += blockDim.x) {
        double lw;
        if (log_w(j, lw)) lmax = fmax(lmax, lw);
    }
    lmax = block_max(lmax, red, nw);
    double tot[2] = {0.0, 0.0};  // sum w, sum w^2 over every model
#pragma unroll
    for (int i = 0; i < kOutCacheW; ++i) {
        if (!c_ok[i]) continue;
        c_w[i] = exp(c_lw[i] - lmax);
        tot[0] += c_w[i];
        tot[1] = fma(c_w[i], c_w[i], tot[1]);
    }
    for (int j = tid + kOutCacheW * (int)blockDim.x; j < n; j += blockDim.x) {
        double lw;
        if (!log_w(j, lw)) continue;
        const double w = exp(lw - lmax);
        tot[0] += w;
        tot[1] = fma(w, w, tot[1]);
    }
    block_sum<2>(tot, red, nw);
    for (int m = 0; m < P.M; ++m) {
        const int kind = P.kinds[m];
        double s1[9];
#pragma unroll
        for (int q = 0; q < 9; ++q) s1[q] = 0.0;
        bool c_m[kOutCacheW];
#pragma unroll
        for (int i = 0; i < kOutCacheW; ++i) {
            const int j = tid + i * (int)blockDim.x;
            c_m[i] = c_ok[i] && ((uint32_t)acc[j] - gb) / P.n_draws == (uint32_t)m;
            if (!c_m[i]) continue;
            bank_slot_values(kind, P.bank_theta + (size_t)(uint32_t)acc[j] * VPET_PSTRIDE, c_val[i]);
#pragma unroll
            for (int q = 0; q < 8; ++q) s1[q] = fma(c_w[i], c_val[i][q], s1[q]);
            s1[8] += c_w[i];
        }
        double val[8];
        for (int j = tid + kOutCacheW * (int)blockDim.x; j < n; j += blockDim.x) {
            double lw;
            const uint32_t g = (uint32_t)acc[j];
            if (!log_w(j, lw) || (g - gb) / P.n_draws != (uint32_t)m) continue;
            const double w = exp(lw - lmax);
            bank_slot_values(kind, P.bank_theta + (size_t)g * VPET_PSTRIDE, val);
#pragma unroll
            for (int q = 0; q < 8; ++q) s1[q] = fma(w, val[q], s1[q]);
            s1[8] += w;
        }
        block_sum<9>(s1, red, nw);
        const double sw = s1[8];
        double mean[8], s2[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            mean[q] = s1[q] / sw;
            s2[q] = 0.0;
        }
#pragma unroll
        for (int i = 0; i < kOutCacheW; ++i) {
            if (!c_m[i]) continue;
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                const double dv = c_val[i][q] - mean[q];
                s2[q] = fma(c_w[i] * dv, dv, s2[q]);
            }
        }
        for (int j = tid + kOutCacheW * (int)blockDim.x; j < n; j += blockDim.x) {
            double lw;
            const uint32_t g = (uint32_t)acc[j];
            if (!log_w(j, lw) || (g - gb) / P.n_draws != (uint32_t)m) continue;
            const double w = exp(lw - lmax);
            bank_slot_values(kind, P.bank_theta + (size_t)g * VPET_PSTRIDE, val);
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                const double dv = val[q] - mean[q];
                s2[q] = fma(w * dv, dv, s2[q]);
            }
        }
        block_sum<8>(s2, red, nw);
        if (tid < 16) {
            const int q = tid >> 1;
            float outv = __builtin_nanf("");
            if (bank_slot_used(kind, q) && sw > 0.0) outv = (tid & 1) == 0 ? (float)mean[q] : (float)(s2[q] / sw);
            P.out_mom[((size_t)orow * P.M + m) * 16 + tid] = outv;
        }
        if (tid == 0) P.out_prob[(size_t)orow * P.M + m] = tot[0] > 0.0 ? (float)(sw / tot[0]) : __builtin_nanf("");
    }
    if (P.out_ess && tid == 0) P.out_ess[orow] = tot[0] > 0.0 ? (float)(tot[0] * tot[0] / tot[1]) : __builtin_nanf("");
}

// bank_outputs_weighted with each accepted key's log weight, weight and bank
// values gathered once into LDS (spare: 5 n free 8-byte slots after the n
// keys): one gather and one exp per key instead of one per pass, the same
// sums in the same order.  A weight of 0 marks a key that takes no part.
__device__ void bank_outputs_weighted_lds(const BankArgs& P, long long row, long long orow, const uint64_t* acc,
                                          double* red, uint64_t* spare) {
    const int n = (int)P.n_acc;
    const int tid = threadIdx.x, nw = blockDim.x >> 6;
    const unsigned gb = bank_row_base(P, row);
    const float h_v = P.below ? P.below[orow] : __builtin_inff();
    double* cw = reinterpret_cast<double*>(spare);    // [n] log weight, then weight
    float* ct = reinterpret_cast<float*>(spare + n);  // [n][8] bank values (16-byte aligned)
    double lmax = -__builtin_inf();
    for (int j = tid; j < n; j += blockDim.x) {
        const uint64_t k = acc[j];
        double lw = -__builtin_inf();
        if (k != kNoKey && __uint_as_float((uint32_t)(k >> 32)) <= h_v) {
            const uint32_t g = (uint32_t)k;
            lw = P.bank_logw[g];
            const float4* src = reinterpret_cast<const float4*>(P.bank_theta + (size_t)g * VPET_PSTRIDE);
            float4* dst = reinterpret_cast<float4*>(ct + (size_t)j * VPET_PSTRIDE);
            dst[0] = src[0];
            dst[1] = src[1];
        }
        cw[j] = lw;
        if (lw > -__builtin_inf()) lmax = fmax(lmax, lw);
    }
    lmax = block_max(lmax, red, nw);
    double tot[2] = {0.0, 0.0};  // sum w, sum w^2 over every model
    for (int j = tid; j < n; j += blockDim.x) {
        const double lw = cw[j];
        double w = 0.0;
        if (lw > -__builtin_inf()) {
            w = exp(lw - lmax);
            tot[0] += w;
            tot[1] = fma(w, w, tot[1]);
        }
        cw[j] = w;
    }
    block_sum<2>(tot, red, nw);
    for (int m = 0; m < P.M; ++m) {
        const int kind = P.kinds[m];
        double s1[9];
#pragma unroll
        for (int q = 0; q < 9; ++q) s1[q] = 0.0;
        double val[8];
        for (int j = tid; j < n; j += blockDim.x) {
            const double w = cw[j];
            if (w == 0.0 || ((uint32_t)acc[j] - gb) / P.n_draws != (uint32_t)m) continue;
            bank_slot_values(kind, ct + (size_t)j * VPET_PSTRIDE, val);
#pragma unroll
            for (int q = 0; q < 8; ++q) s1[q] = fma(w, val[q], s1[q]);
            s1[8] += w;
        }
        block_sum<9>(s1, red, nw);
        const double sw = s1[8];
        double mean[8], s2[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            mean[q] = s1[q] / sw;
            s2[q] = 0.0;
        }
        for (int j = tid; j < n; j += blockDim.x) {
            const double w = cw[j];
            if (w == 0.0 || ((uint32_t)acc[j] - gb) / P.n_draws != (uint32_t)m) continue;
            bank_slot_values(kind, ct + (size_t)j * VPET_PSTRIDE, val);
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                const double dv = val[q] - mean[q];
                s2[q] = fma(w * dv, dv, s2[q]);
            }
        }
        block_sum<8>(s2, red, nw);
        if (tid < 16) {
            const int q = tid >> 1;
            float outv = __builtin_nanf("");
            if (bank_slot_used(kind, q) && sw > 0.0) outv = (tid & 1) == 0 ? (float)mean[q] : (float)(s2[q] / sw);
            P.out_mom[((size_t)orow * P.M + m) * 16 + tid] = outv;
        }
        if (tid == 0) P.out_prob[(size_t)orow * P.M + m] = tot[0] > 0.0 ? (float)(sw / tot[0]) : __builtin_nanf("");
    }
    if (P.out_ess && tid == 0) P.out_ess[orow] = tot[0] > 0.0 ? (float)(tot[0] * tot[0] / tot[1]) : __builtin_nanf("");
}

// Unit-weight outputs with each accepted key's bank values gathered once
// into LDS (spare: 4 n free 8-byte slots after the n keys, 16-byte aligned
// from the second): one gather per key for both moment passes, the same sums
// in the same order.
__device__ void bank_outputs_unit_lds(const BankArgs& P, long long orow, unsigned gb, const uint64_t* acc,
                                      double* red, uint64_t* spare) {
    const int n = (int)P.n_acc;
    const int tid = threadIdx.x;
    float* ct = reinterpret_cast<float*>(spare + (n & 1));  // [n][8] bank values
    for (int j = tid; j < n; j += blockDim.x) {
        const float4* src = reinterpret_cast<const float4*>(P.bank_theta + (size_t)(uint32_t)acc[j] * VPET_PSTRIDE);
        float4* dst = reinterpret_cast<float4*>(ct + (size_t)j * VPET_PSTRIDE);
        dst[0] = src[0];
        dst[1] = src[1];
    }
    for (int m = 0; m < P.M; ++m) {
        const int kind = P.kinds[m];
        double s1[9];
#pragma unroll
        for (int q = 0; q < 9; ++q) s1[q] = 0.0;
        double val[8];
        for (int j = tid; j < n; j += blockDim.x) {
            if (((uint32_t)acc[j] - gb) / P.n_draws != (uint32_t)m) continue;
            bank_slot_values(kind, ct + (size_t)j * VPET_PSTRIDE, val);
#pragma unroll
            for (int q = 0; q < 8; ++q) s1[q] += val[q];
            s1[8] += 1.0;
        }
        block_sum<9>(s1, red, blockDim.x >> 6);
        const double cnt = s1[8];
        double mean[8], s2[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            mean[q] = s1[q] / cnt;
            s2[q] = 0.0;
        }
        for (int j = tid; j < n; j += blockDim.x) {
            if (((uint32_t)acc[j] - gb) / P.n_draws != (uint32_t)m) continue;
            bank_slot_values(kind, ct + (size_t)j * VPET_PSTRIDE, val);
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                const double dv = val[q] - mean[q];
                s2[q] = fma(dv, dv, s2[q]);
            }
        }
        block_sum<8>(s2, red, blockDim.x >> 6);
        if (tid < 16) {
            const int q = tid >> 1;
            float outv = __builtin_nanf("");
            if (bank_slot_used(kind, q) && cnt > 0.0) {
                if ((tid & 1) == 0)
                    outv = (float)mean[q];
                else
                    outv = (cnt > 1.0) ? (float)(s2[q] / (cnt - 1.0)) : 0.0f;
            }
            P.out_mom[((size_t)orow * P.M + m) * 16 + tid] = outv;
        }
        if (tid == 0) P.out_prob[(size_t)orow * P.M + m] = (float)(cnt / (double)n);
    }
}

// Outputs of one voxel from its n accepted keys (sorted, in LDS).  MODE 0:
// unit row weights, 1: the bank's importance weights, 2: whichever the launch
// has (one instance per mode keeps the select kernels' registers to what
// their path needs).
// spare (MODES 0, 1): LDS past the keys for the staged outputs.
template <int MODE>
__device__ void bank_outputs_m(const BankArgs& P, long long row, const uint64_t* acc, double* red,
                               uint64_t* spare = nullptr) {
    const int n = (int)P.n_acc;
    const int tid = threadIdx.x;
    const long long orow = bank_out_row(P, row);
    const unsigned gb = bank_row_base(P, row);
    if (P.out_idx)  // rows of the voxel's own bank
        for (int j = tid; j < n; j += blockDim.x) P.out_idx[(size_t)orow * n + j] = (int)((uint32_t)acc[j] - gb);
    if (P.out_dist)
        for (int j = tid; j < n; j += blockDim.x)
            P.out_dist[(size_t)orow * n + j] = __uint_as_float((uint32_t)(acc[j] >> 32));
    if (P.out_thr && tid == 0) P.out_thr[orow] = __uint_as_float((uint32_t)(acc[n - 1] >> 32));
    if (MODE == 1) {
        bank_outputs_weighted_lds(P, row, orow, acc, red, spare);
        return;
    }
    if (MODE == 2 && P.bank_logw) {
        bank_outputs_weighted(P, row, orow, acc, red);
        return;
    }
    if (MODE == 0) {
        bank_outputs_unit_lds(P, orow, gb, acc, red, spare);
        return;
    }
    for (int m = 0; m < P.M; ++m) {
        const int kind = P.kinds[m];
        double s1[9];
#pragma unroll
        for (int q = 0; q < 9; ++q) s1[q] = 0.0;
        // the first kOutCache keys of this thread keep their values in
        // registers for the second pass (the same sums in the same order)
        double c_val[kOutCache][8];
        bool c_m[kOutCache];
#pragma unroll
        for (int i = 0; i < kOutCache; ++i) {
            const int j = tid + i * (int)blockDim.x;
            c_m[i] = j < n && ((uint32_t)acc[j] - gb) / P.n_draws == (uint32_t)m;
            if (!c_m[i]) continue;
            bank_slot_values(kind, P.bank_theta + (size_t)(uint32_t)acc[j] * VPET_PSTRIDE, c_val[i]);
#pragma unroll
            for (int q = 0; q < 8; ++q) s1[q] += c_val[i][q];
            s1[8] += 1.0;
        }
        double val[8];
        for (int j = tid + kOutCache * (int)blockDim.x; j < n; j += blockDim.x) {
            const uint32_t g = (uint32_t)acc[j];
            if ((g - gb) / P.n_draws != (uint32_t)m) continue;
            bank_slot_values(kind, P.bank_theta + (size_t)g * VPET_PSTRIDE, val);
#pragma unroll
            for (int q = 0; q < 8; ++q) s1[q] += val[q];
            s1[8] += 1.0;
        }
        block_sum<9>(s1, red, blockDim.x >> 6);
        const double cnt = s1[8];
        double mean[8], s2[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            mean[q] = s1[q] / cnt;
            s2[q] = 0.0;
        }
#pragma unroll
        for (int i = 0; i < kOutCache; ++i) {
            if (!c_m[i]) continue;
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                const double dv = c_val[i][q] - mean[q];
                s2[q] = fma(dv, dv, s2[q]);
            }
        }
        for (int j = tid + kOutCache * (int)blockDim.x; j < n; j += blockDim.x) {
            const uint32_t g = (uint32_t)acc[j];
            if ((g - gb) / P.n_draws != (uint32_t)m) continue;
            bank_slot_values(kind, P.bank_theta + (size_t)g * VPET_PSTRIDE, val);
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                const double dv = val[q] - mean[q];
                s2[q] = fma(dv, dv, s2[q]);
            }
        }
        block_sum<8>(s2, red, blockDim.x >> 6);
        if (tid < 16) {
            const int q = tid >> 1;
            float outv = __builtin_nanf("");
            if (bank_slot_used(kind, q) && cnt > 0.0) {
                if ((tid & 1) == 0)
                    outv = (float)mean[q];
                else
                    outv = (cnt > 1.0) ? (float)(s2[q] / (cnt - 1.0)) : 0.0f;
            }
            P.out_mom[((size_t)orow * P.M + m) * 16 + tid] = outv;
        }
        if (tid == 0) P.out_prob[(size_t)orow * P.M + m] = (float)(cnt / (double)n);
    }
}

__device__ __forceinline__ void bank_outputs(const BankArgs& P, long long row, const uint64_t* acc, double* red) {
    bank_outputs_m<2>(P, row, acc, red);
}

__device__ void bank_invalid(const BankArgs& P, long long row) {
    const int n = (int)P.n_acc;
    const float qnan = __builtin_nanf("");
    const long long orow = bank_out_row(P, row);
    for (int j = threadIdx.x; j < P.M * 16; j += blockDim.x) P.out_mom[(size_t)orow * P.M * 16 + j] = qnan;
    for (int j = threadIdx.x; j < P.M; j += blockDim.x) P.out_prob[(size_t)orow * P.M + j] = qnan;
    if (P.out_idx)
        for (int j = threadIdx.x; j < n; j += blockDim.x) P.out_idx[(size_t)orow * n + j] = -1;
    if (P.out_dist)
        for (int j = threadIdx.x; j < n; j += blockDim.x) P.out_dist[(size_t)orow * n + j] = qnan;
    if (P.out_thr && threadIdx.x == 0) P.out_thr[orow] = qnan;
    if (P.out_ess && threadIdx.x == 0) P.out_ess[orow] = qnan;
}

// Ascending sort of one 64-bit value per lane across the wavefront (bitonic;
// lane l ends with the l-th smallest).
__device__ __forceinline__ uint64_t wave_sort_lanes(uint64_t x) {
    const int lane = lane_id();
#pragma unroll
    for (int k = 2; k <= kWave; k <<= 1) {
#pragma unroll
        for (int j = k >> 1; j > 0; j >>= 1) {
            const uint32_t lo = (uint32_t)__shfl_xor((int)(uint32_t)x, j, kWave);
            const uint32_t hi = (uint32_t)__shfl_xor((int)(uint32_t)(x >> 32), j, kWave);
            const uint64_t y = ((uint64_t)hi << 32) | lo;
            const bool lower = (lane & j) == 0, up = (lane & k) == 0;
            x = (lower == up) ? (x < y ? x : y) : (x < y ? y : x);
        }
    }
    return x;
}

// Moves the m <= below smallest of the wavefront's `below` distinct keys in
// LDS to the front and returns m, with n <= m: a pivot taken from 64 evenly
// spaced keys, at about 1.25 n of them below it, is checked by counting and
// raised until at least n keys lie at or below it (else every key stays).
// The n smallest keys are then among the first m, in fewer to sort.
__device__ __forceinline__ int keep_smallest(uint64_t* keys, int below, int n, uint64_t* cut = nullptr) {
    const int lane = lane_id();
    wave_lds_sync();
    const uint64_t smp = wave_sort_lanes(keys[(int)(((long long)lane * below) / kWave)]);
    int q = (int)min(63LL, (64LL * (n + n / 4) + below - 1) / below);
    for (int attempt = 0; attempt < 3; ++attempt) {
        const uint64_t piv = ((uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(smp >> 32), q) << 32) |
                             (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)smp, q);
        int cnt = 0;
        for (int j0 = 0; j0 < below; j0 += kWave) {
            const int j = j0 + lane;
            cnt += __popcll(__ballot(j < below && keys[j] <= piv));
        }
        if (cnt >= n) {
            int m = 0;  // each chunk is read before it is written, at lower indices
            for (int j0 = 0; j0 < below; j0 += kWave) {
                const int j = j0 + lane;
                const uint64_t k = j < below ? keys[j] : kNoKey;
                const bool in = j < below && k <= piv;
                const uint64_t b = __ballot(in);
                wave_lds_sync();
                if (in) keys[m + (int)mbcnt(b)] = k;
                m += __popcll(b);
                wave_lds_sync();
            }
            if (cut) *cut = piv;
            return m;
        }
        if (q == kWave - 1) break;
        q = min(kWave - 1, q + (8 << attempt));
    }
    return below;
}

// One wavefront per voxel: sort the candidates, keep the n smallest.  With
// RECOMPUTE the candidates carry only their bank row and the exact FP64
// distance is computed here.  The result is certified when at least n
// candidates have fp32 distance <= the pilot threshold (every bank row below
// the threshold is a candidate, so the n smallest keys are among them);
// otherwise -- or when the buffer overflowed -- the voxel is marked for the
// exact fallback.
template <int LD, bool L1, bool RECOMPUTE, bool WEIGHTED>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(4))) void vpet_bank_select_kernel(BankArgs P) {
    extern __shared__ __align__(16) unsigned char lds[];
    uint64_t* keys = reinterpret_cast<uint64_t*>(lds);
    double* red = reinterpret_cast<double*>(keys + (RECOMPUTE ? P.scap : P.cap));
    double* Ys = red + kRedStride * kMaxWpv;  // RECOMPUTE: the voxel's curve and weights
    double* Ws = Ys + LD;
    const long long row = blockIdx.x;
    if (row >= P.V) return;
    // the voxel's scalars and (RECOMPUTE) its TAC value of this lane's frame,
    // loaded together: the kernel is bound by the latency of such round trips
    const int c = P.cnt[row];
    const int c_hi = RECOMPUTE ? P.cnt_hi[row] : 0;
    const float tau = P.tau[row];
    const float tau1 = RECOMPUTE ? P.tau1[row] : 0.0f, cthr1 = RECOMPUTE ? P.cthr1[row] : 0.0f;
    const float y_lane = (RECOMPUTE && lane_id() < P.F) ? P.tacs[(size_t)row * P.F + lane_id()] : 0.0f;
    if (c < 0) {
        bank_invalid(P, row);
        return;
    }
    if (c < (int)P.n_acc || c > P.cap) {
        if (threadIdx.x == 0) P.fb_list[atomicAdd(P.fb_count, 1u)] = (int)row;
        return;
    }
    int below = 0;
    if (RECOMPUTE) {
        // Exact FP64 distances of the candidate rows, keys up to tau packed to
        // the front.  Pass 1 takes the rows that passed the tighter test
        // (computed S <= cthr1); if at least n of them lie at or below tau1,
        // the n smallest keys are among them.  Otherwise pass 2 adds the
        // remaining candidates and the certificate is taken at tau.  Taken
        // rows queue up in LDS; a batch of up to 64 is ranked 16 rows at a
        // time, four lanes per row, each lane a quarter of the frames
        // (16-byte loads of whole row segments).
        wave_curve_lds<LD, L1>(P, row, y_lane, Ys, Ws);
        uint32_t* queue = reinterpret_cast<uint32_t*>(Ws + LD);  // 2 x 64 rows
        const uint64_t* src = P.cand + (size_t)row * P.cap;
        const int c0 = c - c_hi;
        const int lane = lane_id(), part = lane & 3;
        constexpr int Q = LD / 4;
        double Yq[Q], Wq[Q];  // this lane's quarter of the curve and weights
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            Yq[q] = Ys[part * Q + q];
            Wq[q] = Ws[part * Q + q];
        }
        int below1 = 0, queued = 0;
        bool overflow = false;  // more keys at or below tau than the LDS holds: exact fallback
        // Keys above `cut` cannot be among the n smallest: when a round could
        // overflow the buffer it first keeps only the keys at or below a pivot
        // with at least n of them at or below it (keep_smallest), and later
        // keys above that pivot are dropped; it overflows only if that fails.
        uint64_t cut = kNoKey;
        auto rank = [&](int nb) {  // queue[0, nb), nb <= 64: 32 rows per round, their loads issued together
            for (int i0 = 0; i0 < nb; i0 += 32) {
                // a round adds at most 32 keys
                if (!overflow && below > P.scap - 32) below = keep_smallest(keys, below, (int)P.n_acc, &cut);
                uint32_t g[2];
                double xv[2][Q];
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    const int i = i0 + 16 * h + (lane >> 2);
                    g[h] = queue[i < nb ? i : 0];
                    const double* xr = static_cast<const double*>(
                        __builtin_assume_aligned(P.bank_x + (size_t)g[h] * LD + part * Q, 16));
#pragma unroll
                    for (int q = 0; q < Q; ++q) xv[h][q] = xr[q];
                }
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    const bool live = i0 + 16 * h + (lane >> 2) < nb;
                    double pt = 0.0;
#pragma unroll
                    for (int q = 0; q < Q; ++q) pt = dist_term<L1>(Yq[q], Wq[q], xv[h][q], pt);
                    pt += dpp_f64<0xB1>(pt);  // p0 + p1, p2 + p3 (quad_perm [1,0,3,2])
                    pt += dpp_f64<0x4E>(pt);  // (p0 + p1) + (p2 + p3) (quad_perm [2,3,0,1])
                    const float fd = key_dist(pt);
                    const bool mine = live && part == 0;
                    const uint64_t key = ((uint64_t)__float_as_uint(fd) << 32) | g[h];
                    const bool keep = mine && fd <= tau && key <= cut;
                    const uint64_t b = __ballot(keep);
                    overflow = overflow || below + __popcll(b) > P.scap;
                    if (keep && !overflow) keys[below + (int)mbcnt(b)] = key;
                    below += __popcll(b);
                    below1 += __popcll(__ballot(mine && fd <= tau1));
                }
            }
        };
        for (int pass = 0; pass < 2; ++pass) {
            for (int j0 = 0; j0 < c; j0 += 4 * kWave) {
                uint64_t e[4];  // four list entries per lane, loaded together
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const int j = j0 + u * kWave + lane;
                    e[u] = j < c ? src[cand_slot(P, j, c0)] : 0ull;
                }
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const bool take = j0 + u * kWave + lane < c &&
                                      (__uint_as_float((uint32_t)(e[u] >> 32)) <= cthr1) == (pass == 0);
                    const uint64_t b = __ballot(take);
                    if (take) queue[queued + (int)mbcnt(b)] = (uint32_t)e[u];  // queued < 64 here
                    queued += __popcll(b);
                    wave_lds_sync();
                    if (queued >= kWave) {
                        rank(kWave);
                        queued -= kWave;
                        const uint32_t rest = lane < queued ? queue[kWave + lane] : 0u;
                        wave_lds_sync();
                        if (lane < queued) queue[lane] = rest;
                        wave_lds_sync();
                    }
                }
            }
            if (queued > 0) {
                rank(queued);
                queued = 0;
            }
            if (below1 >= (int)P.n_acc) break;  // certified at tau1
        }
        if (overflow) {
            if (threadIdx.x == 0) P.fb_list[atomicAdd(P.fb_count, 1u)] = (int)row;
            return;
        }
        if (below1 >= (int)P.n_acc) {
            // certified at tau1: only the keys at or below tau1 can be among
            // the n smallest, so they alone are moved to the front and sorted
            // (each chunk is read before it is written, at lower indices)
            int m = 0;
            for (int j0 = 0; j0 < below; j0 += kWave) {
                const int j = j0 + lane;
                const uint64_t k = j < below ? keys[j] : kNoKey;
                const bool in = j < below && __uint_as_float((uint32_t)(k >> 32)) <= tau1;
                const uint64_t b = __ballot(in);
                wave_lds_sync();
                if (in) keys[m + (int)mbcnt(b)] = k;
                m += __popcll(b);
                wave_lds_sync();
            }
            below = m;
        }
    } else {
        const uint64_t* src = P.cand + (size_t)row * P.cap;
        const int c0 = c - P.cnt_hi[row];
        for (int j = lane_id(); j < c; j += kWave) keys[j] = src[cand_slot(P, j, c0)];
        below = c;
    }
    if (below < (int)P.n_acc) {
        if (threadIdx.x == 0) P.fb_list[atomicAdd(P.fb_count, 1u)] = (int)row;
        return;
    }
    if (below > 2 * (int)P.n_acc) below = keep_smallest(keys, below, (int)P.n_acc);
    const int len = below <= 1 ? 2 : (1 << (32 - __clz(below - 1)));
    for (int j = below + lane_id(); j < len; j += kWave) keys[j] = kNoKey;
    wave_lds_sync();
    wave_bitonic_sort(keys, len);
    // the accepted keys' values (and weights) are staged in the LDS past the n
    // accepted keys (scap >= 6 n with weights, >= 5 n + 1 without)
    bank_outputs_m<WEIGHTED ? 1 : 0>(P, row, keys, red, keys + P.n_acc);
}

// Exact fallback: one block per listed voxel streams every bank row; each
// wavefront keeps a running top-n of its share of the rows (the per-voxel
// selection of the infer kernel, in fb_cap keys), and a block-wide bitonic
// sort merges the shares.  A fixed grid walks the list, whose length the
// select kernel left in fb_count.
template <int LD, bool L1>
__global__ __launch_bounds__(512) void vpet_bank_fallback_kernel(BankArgs P) {
    extern __shared__ __align__(16) unsigned char lds[];
    const int nw = blockDim.x >> 6, wave = threadIdx.x >> 6;
    uint64_t* keys_all = reinterpret_cast<uint64_t*>(lds);
    double* red = reinterpret_cast<double*>(keys_all + (size_t)nw * P.fb_cap);
    const unsigned n_fb = *P.fb_count;
    for (unsigned item = blockIdx.x; item < n_fb; item += gridDim.x) {
        const long long row = P.fb_list[item];
        double Y[LD], Wt[LD];
        lane_curve<LD, L1>(P, row, Y, Wt);  // every lane holds the same voxel
        TopN top;
        top.keys = keys_all + (size_t)wave * P.fb_cap;
        top.n = (int)P.n_acc;
        top.cap = P.fb_cap;
        top.nbuf = 0;
        top.tau = kNoKey;
        __syncthreads();  // the previous voxel's outputs have read the keys
        for (int j = lane_id(); j < P.fb_cap; j += kWave) top.keys[j] = kNoKey;
        wave_lds_sync();
        const unsigned gb = bank_row_base(P, row);
        for (unsigned g0 = (unsigned)wave * kWave; g0 < P.n_tot; g0 += (unsigned)nw * kWave) {
            const unsigned g = g0 + (unsigned)lane_id();
            uint64_t key[1] = {kNoKey};
            if (g < P.n_tot) {
                const float fd = key_dist(row_distance<LD, L1>(P.bank_x + (size_t)(gb + g) * LD, Y, Wt));
                key[0] = ((uint64_t)__float_as_uint(fd) << 32) | (gb + g);
            }
            top.insert(key);
        }
        top.merge();
        __syncthreads();
        if (nw > 1) block_bitonic_sort(keys_all, nw * P.fb_cap);
        bank_outputs(P, row, keys_all, red);
    }
}

__global__ void vpet_bank_reset_kernel(BankArgs P) {
    if (blockIdx.x == 0 && threadIdx.x == 0) *P.fb_count = 0u;
}

// vpet_abc_bank_screen: every valid voxel's candidate test admits every row
// (the operand kernel has marked invalid voxels with a_v = NaN).
__global__ __launch_bounds__(256) void vpet_bank_passall_kernel(BankArgs P) {
    const long long v = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= P.V) return;
    const double a = P.aval[v];
    P.cthr[v] = a == a ? __builtin_inff() : -__builtin_inff();
    P.cnt[v] = a == a ? 0 : -1;
    P.cnt_hi[v] = 0;
}

// vpet_abc_bank_screen: voxel `blockIdx.x`'s candidates (computed S, bank row)
// scattered to out_s[v][row]; rows never listed (invalid voxel) stay NaN.
__global__ __launch_bounds__(256) void vpet_bank_scatter_kernel(BankArgs P, float* out_s, double* out_a) {
    const long long v = blockIdx.x;
    float* dst = out_s + (size_t)v * P.n_tot;
    for (unsigned j = threadIdx.x; j < P.n_tot; j += blockDim.x) dst[j] = __builtin_nanf("");
    if (threadIdx.x == 0) out_a[v] = P.aval[v];
    __syncthreads();
    const int c = P.cnt[v];
    const int c0 = c - P.cnt_hi[v];
    const uint64_t* src = P.cand + (size_t)v * P.cap;
    for (int j = threadIdx.x; j < c && j < P.cap; j += blockDim.x) {
        const uint64_t e = src[cand_slot(P, j, c0)];
        const uint32_t g = (uint32_t)e;
        if (g < P.n_tot) dst[g] = __uint_as_float((uint32_t)(e >> 32));
    }
}

// --- BF16 contraction -------------------------------------------------------
typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8_t;
typedef __attribute__((__vector_size__(16 * sizeof(float)))) float f32x16_t;
constexpr int kMfmaVox = 256;  // voxels per block: 8 wavefronts x 32 rows
constexpr int kMfmaRows = 32;  // bank rows per tile
constexpr int kScreenMaxRows = 4096;     // vpet_abc_bank_screen: bank rows (the largest candidate list)
constexpr int kScreenMaxVoxels = 1 << 16;

__device__ __forceinline__ uint16_t bf16_rn(float f) {  // round to nearest even
    const uint32_t u = __float_as_uint(f);
    return (uint16_t)((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
}
__device__ __forceinline__ float bf16_to_f(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }

__device__ __forceinline__ void split_bf16(double v, uint16_t& hi, uint16_t& lo) {
    hi = bf16_rn((float)v);
    lo = bf16_rn((float)(v - (double)bf16_to_f(hi)));
}

// split_bf16 of two values at once, packed (first value in the low half), with
// gfx950's paired conversion (v_cvt_pk_bf16_f32, round to nearest even: the
// same bits as bf16_rn for every non-NaN value).
typedef float vpet_f32x2 __attribute__((ext_vector_type(2)));
typedef __bf16 vpet_bf16x2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ uint32_t bf16x2_rn(float a, float b) {
    const vpet_f32x2 v = {a, b};
    return __builtin_bit_cast(uint32_t, __builtin_convertvector(v, vpet_bf16x2));
}
__device__ __forceinline__ void split_bf16x2(double v0, double v1, uint32_t& hi, uint32_t& lo) {
    hi = bf16x2_rn((float)v0, (float)v1);
    lo = bf16x2_rn((float)(v0 - (double)__uint_as_float(hi << 16)),
                   (float)(v1 - (double)__uint_as_float(hi & 0xFFFF0000u)));
}

// A row of 2 LD bf16 values (LD words) written as 16-byte stores.
template <int LD>
__device__ __forceinline__ void store_words(uint16_t* dst, const uint32_t (&w)[LD]) {
    uint4* d = reinterpret_cast<uint4*>(dst);
#pragma unroll
    for (int q = 0; q < LD / 4; ++q) d[q] = make_uint4(w[4 * q], w[4 * q + 1], w[4 * q + 2], w[4 * q + 3]);
}

// Bank operands B_g = [x_g, x_g^2] as bf16 hi/lo parts (x_g - r and its
// square with a group reference curve r: the distance is unchanged, since
// d = sum w ((y - r) - (x - r))^2, while the screen's operands and hence its
// error bound shrink to the size of the deviations from r).
template <int LD>
// A thread per pair of frames of a row (coalesced 16-byte reads, 4-byte
// writes of bf16 pairs).
__global__ __launch_bounds__(256) void vpet_bank_bops_kernel(BankArgs P) {
    const unsigned long long t = (unsigned long long)blockIdx.x * blockDim.x + threadIdx.x;
    const unsigned long long g = t / (LD / 2);
    if (g >= P.n_tot) return;
    const int f = 2 * (int)(t - g * (LD / 2));
    const double2 x2 = *reinterpret_cast<const double2*>(P.bank_x + g * LD + f);
    double x0 = x2.x, x1 = x2.y;
    if (P.ref) {
        const double* rr = P.ref + (size_t)(g / P.grp_rows) * LD + f;
        x0 -= rr[0];
        x1 -= rr[1];
    }
    uint32_t* bh = reinterpret_cast<uint32_t*>(P.bhi + g * 2 * LD);
    uint32_t* bl = reinterpret_cast<uint32_t*>(P.blo + g * 2 * LD);
    split_bf16x2(x0, x1, bh[f / 2], bl[f / 2]);
    split_bf16x2(x0 * x0, x1 * x1, bh[(LD + f) / 2], bl[(LD + f) / 2]);
}

// Voxel operands A_v = [-2 w y, w] (bf16 hi/lo) and a_v = sum w y^2 (FP64),
// so that d_vg = a_v + sum_k A_vk B_gk (with a group reference curve r, y - r
// in place of y and x - r in place of x).  An invalid voxel gets zero operands,
// a_v = NaN, threshold NaN and count -1.
template <int LD>
__global__ __launch_bounds__(256) void vpet_bank_aops_kernel(BankArgs P) {
    const long long row = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (row >= P.V) return;
    double Y[LD], Wt[LD];
    const bool valid = lane_curve<LD, false>(P, row, Y, Wt);
    if (P.ref) {
        const double* rr =
            P.ref + (size_t)((unsigned long long)(P.pos0 + row) / P.grp_vox - (unsigned long long)P.g0) * LD;
#pragma unroll
        for (int f = 0; f < LD; ++f) Y[f] -= rr[f];
    }
    uint16_t* ah = P.ahi + (size_t)row * 2 * LD;
    uint16_t* al = P.alo + (size_t)row * 2 * LD;
    uint32_t wh[LD], wl[LD];  // K = 2 LD bf16 values, two per word
    if (!valid) {
#pragma unroll
        for (int q = 0; q < LD; ++q) wh[q] = wl[q] = 0u;
        store_words<LD>(ah, wh);
        store_words<LD>(al, wl);
        P.aval[row] = __builtin_nan("");
        P.tau[row] = P.tau1[row] = __builtin_nanf("");
        P.cthr[row] = P.cthr1[row] = -__builtin_inff();
        P.cnt[row] = -1;
        return;
    }
    double a = 0.0;
    bool wneg = false;
#pragma unroll
    for (int k = 0; k < 2 * LD; ++k) {
        const int f = k < LD ? k : k - LD;
        if (k < LD) {
            a = fma(Wt[f] * Y[f], Y[f], a);
            wneg = wneg || !(Wt[f] >= 0.0);
        }
        uint16_t hi, lo;
        split_bf16(k < LD ? -2.0 * Wt[f] * Y[f] : Wt[f], hi, lo);
        if (k & 1) {
            wh[k >> 1] |= (uint32_t)hi << 16;
            wl[k >> 1] |= (uint32_t)lo << 16;
        } else {
            wh[k >> 1] = hi;
            wl[k >> 1] = lo;
        }
    }
    store_words<LD>(ah, wh);
    store_words<LD>(al, wl);
    // the error bound assumes w >= 0: otherwise a_v = -inf makes every row a
    // candidate (the selection is then exact or falls back)
    P.aval[row] = wneg ? -__builtin_inf() : a;
}

// Error of the split contraction.  With A = A_hi + A_lo + e_A (|A_lo| and
// |e_A|/|A_hi + A_lo| at most 2^-8 and 2^-16 relative) and likewise B, the sum
// of the three products hi*hi + hi*lo + lo*hi differs from sum_k A_k B_k by the
// dropped lo*lo product and the two residual terms, at most 3 * 2^-16 * E with
// E = sum_k |A_k||B_k|; the products of bf16 values are exact in FP32 and
// their FP32 accumulation (3K terms) adds at most 3K * 2^-24 * E under round to
// nearest.  The factor 2 covers truncating accumulation in the matrix cores and
// the second-order terms.
template <int K>
__host__ __device__ constexpr double contraction_rel_err() {
    return 2.0 * (3.0 * 0x1p-16 + 3.0 * K * 0x1p-24);
}

// One block = 256 voxels (8 wavefronts, 32 each) against the bank, in tiles of
// 64 rows staged in LDS (double-buffered; the global loads of tile t+2 are
// issued while tile t is multiplied and land in LDS one tile later; two
// independent 32-row accumulators per wavefront).  Per tile and k-step a
// wavefront issues v_mfma_f32_32x32x16_bf16 on the hi/lo parts, the bank rows
// as the first operand and its voxels as the second: hi*hi + hi*lo + lo*hi
// gives S ~ sum_k A B.  Result r of lane l is then voxel l % 32 of the
// wavefront against row 8 (r/4) + 4 (l/32) + r%4 of the 32-row half: a lane
// serves one voxel, and its two half-wavefronts see 16 of every 32 rows each.
//
// PILOT (n_pilot rows, taken from tiles spread evenly over the bank, which is
// ordered by model): for each of its 16 results a lane keeps the minimum of S
// over that result's rows (one class of rows mod 32), so a voxel's 32 class
// minima sit in lanes l and l + 32; the 16th smallest of them, plus a_v, is
// its threshold tau_v (rounded to fp32).  With n_pilot = 5.5 N / n about 4 n
// bank rows fall below tau_v (order statistics of the class minima); tau_v
// only steers the work -- the selection certifies or falls back.  The
// candidate threshold is
//   cthr_v = tau_v - a_v + m E_tau + 1e-6 (a_v + |tau_v|),
// m = contraction_rel_err, E_tau = 3 a_v + 4 sqrt(a_v tau_v) + tau_v: for any
// pair with exact distance d <= tau_v, |x| <= |y| + |y - x| and Cauchy-Schwarz
// give E = sum w (2|y||x| + x^2) <= 3 a_v + 4 sqrt(a_v d) + d <= E_tau, so its
// computed S is at most S + m E_tau <= cthr_v; the last term covers the fp32
// roundings of tau_v, a_v and cthr_v.
//
// SCAN (every row): a (voxel, row) pair is a candidate when S <= cthr_v, so
// every row whose exact distance is <= tau_v is a candidate.  A voxel's list
// has two halves of cap / 2 entries, one per half-wavefront: each lane appends
// its voxel's candidates to its own half with a count in a register, so a
// candidate costs no cross-lane work.  cnt = both halves' count (cap + 1 when
// either half overflowed), cnt_hi = the second half's.
template <int K, bool PILOT>
__device__ __forceinline__ void bank_mfma_body(const BankArgs& P) {
    constexpr int KS = K / 16;
    constexpr int RS = 2 * K + 16;        // LDS row stride (bytes), padded against bank conflicts
    constexpr int TR = 2 * kMfmaRows;     // bank rows per tile: two 32-row halves
    constexpr int CA = TR * K / 8;        // 16-byte chunks per array (hi or lo) per tile
    constexpr int CPT = (2 * CA + 511) / 512;  // chunks per thread and tile
    static_assert(CA % 64 == 0 && CPT <= 3, "whole wavefronts per array, at most three chunks per thread");
    __shared__ __align__(16) unsigned char tile[2][2][TR * RS];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const unsigned half = (unsigned)lane >> 5;
    const long long vbase = (long long)blockIdx.x * kMfmaVox;
    const unsigned gb = bank_row_base(P, vbase);  // the block's bank (groups hold whole 256-voxel tiles)

    // this lane's voxel; its operand is the second MFMA operand (k = 16 ks + 8 half + e)
    const long long v = vbase + wave * 32 + (lane & 31);
    bf16x8_t ah[KS], al[KS];
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
        uint4 h = make_uint4(0, 0, 0, 0), l = make_uint4(0, 0, 0, 0);
        if (v < P.V) {
            const size_t off = (size_t)v * K + ks * 16 + half * 8;
            h = *reinterpret_cast<const uint4*>(P.ahi + off);
            l = *reinterpret_cast<const uint4*>(P.alo + off);
        }
        ah[ks] = __builtin_bit_cast(bf16x8_t, h);
        al[ks] = __builtin_bit_cast(bf16x8_t, l);
    }
    // SCAN: the voxel's candidate threshold.  PILOT: per result, the running
    // minimum of S over its class of rows.
    const float cth = PILOT ? 0.0f : (v < P.V ? P.cthr[v] : -__builtin_inff());
    float cmin[PILOT ? 16 : 1];
#pragma unroll
    for (int r = 0; r < (PILOT ? 16 : 1); ++r) cmin[r] = __builtin_inff();
    // SCAN: this lane's half of its voxel's list, as byte offsets from the
    // block's first list (256 lists of at most 8192 entries: 32 bits suffice):
    // its start, its last entry and the next free entry
    const unsigned hcap = (unsigned)P.cap >> 1;
    unsigned char* blist = reinterpret_cast<unsigned char*>(P.cand + (size_t)vbase * (size_t)P.cap);
    const unsigned loff = ((unsigned)(wave * 32 + (lane & 31)) * (unsigned)P.cap + half * hcap) * 8u;
    const unsigned llast = loff + (hcap - 1u) * 8u;
    unsigned lnext = loff;

    // PILOT: ceil(n_pilot / TR) tiles spread evenly over the bank (it is
    // ordered by model, so a prefix would see one model only)
    const unsigned n_rows = P.n_tot;
    const unsigned all_tiles = (n_rows + TR - 1) / TR;
    const unsigned pilot_tiles = (P.n_pilot + TR - 1) / TR;
    const unsigned ntiles = (PILOT && pilot_tiles < all_tiles) ? pilot_tiles : all_tiles;
    auto tile_row0 = [&](unsigned t) {
        return (PILOT ? (unsigned)(((uint64_t)t * all_tiles) / ntiles) : t) * (unsigned)TR;
    };
    // this thread's 16-byte chunks of a tile: array (hi/lo; CA is a multiple of
    // 64, so the array is the same for the whole wavefront), row, column
    const uint16_t* c_src[CPT];
    int c_row[CPT], c_dst[CPT];
    bool c_has[CPT], c_hi[CPT];
#pragma unroll
    for (int u = 0; u < CPT; ++u) {
        const int c = tid + 512 * u;
        c_has[u] = c < 2 * CA;
        const int arr = __builtin_amdgcn_readfirstlane(c / CA), rem = c - arr * CA;
        c_hi[u] = arr == 0;
        c_row[u] = rem / (K / 8);
        const int col = rem - c_row[u] * (K / 8);
        c_src[u] = (arr ? P.blo : P.bhi) + col * 8;
        c_dst[u] = arr * TR * RS + c_row[u] * RS + col * 16;
    }
    uint4 pre[CPT];
    auto fetch = [&](unsigned t) {
#pragma unroll
        for (int u = 0; u < CPT; ++u) {
            const unsigned g = tile_row0(t) + c_row[u];
            // rows past the bank: NaN hi parts, so that their products never pass a test
            const uint32_t pad = c_hi[u] ? 0x7FC07FC0u : 0u;
            pre[u] = make_uint4(pad, pad, pad, pad);
            if (c_has[u] && g < n_rows) pre[u] = *reinterpret_cast<const uint4*>(c_src[u] + (size_t)(gb + g) * K);
        }
    };
    auto stash = [&](int buf) {
#pragma unroll
        for (int u = 0; u < CPT; ++u)
            if (c_has[u]) *reinterpret_cast<uint4*>(&tile[buf][0][0] + c_dst[u]) = pre[u];
    };
    // screen one 32-row half starting at bank row g0 (j0: its position in the
    // pilot sample); result r is row g0 + 8 (r/4) + 4 half + r%4
    auto screen = [&](const f32x16_t& acc, unsigned g0, unsigned j0) {
        if (PILOT) {
            // (rows past the bank compute NaN, which fminf ignores)
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const unsigned o = 8u * (r >> 2) + 4u * half + (r & 3);
                if (j0 + o < P.n_pilot) cmin[r] = fminf(cmin[r], acc[r]);
            }
            return;
        }
        const unsigned grow = gb + g0 + 4u * half;
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            if (acc[r] <= cth) {
                // past the end of the half the last entry is overwritten: the
                // count reports the overflow
                *reinterpret_cast<uint64_t*>(blist + min(lnext, llast)) =
                    ((uint64_t)__float_as_uint(acc[r]) << 32) | (grow + 8u * (r >> 2) + (r & 3));
                lnext += 8u;
            }
        }
    };
    fetch(0);
    stash(0);
    if (ntiles > 1) fetch(1);
    __syncthreads();
    for (unsigned t = 0; t < ntiles; ++t) {
        const int buf = t & 1;
        // while a wavefront copies a tile and issues its products it goes
        // before the others' screens (measured: 3-4 % off the K <= 64 scans,
        // but 22 % slower for the K = 80 one, which keeps the default order)
        if constexpr (K <= 64) __builtin_amdgcn_s_setprio(1);
        if (t + 1 < ntiles) {
            // tile t+1 (fetched one iteration ago) into the other buffer, which
            // every wave finished reading before the last barrier
            stash(buf ^ 1);
            if (t + 2 < ntiles) fetch(t + 2);
        }
        f32x16_t acc0 = {}, acc1 = {};
#pragma unroll
        for (int ks = 0; ks < KS; ++ks) {
            const int off = (lane & 31) * RS + (ks * 16 + half * 8) * 2;
            const unsigned char* hi = &tile[buf][0][0];
            const unsigned char* lo = hi + TR * RS;
            const bf16x8_t bh0 = __builtin_bit_cast(bf16x8_t, *reinterpret_cast<const uint4*>(hi + off));
            const bf16x8_t bl0 = __builtin_bit_cast(bf16x8_t, *reinterpret_cast<const uint4*>(lo + off));
            const bf16x8_t bh1 = __builtin_bit_cast(bf16x8_t, *reinterpret_cast<const uint4*>(hi + 32 * RS + off));
            const bf16x8_t bl1 = __builtin_bit_cast(bf16x8_t, *reinterpret_cast<const uint4*>(lo + 32 * RS + off));
            acc0 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(bh0, ah[ks], acc0, 0, 0, 0);
            acc1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(bh1, ah[ks], acc1, 0, 0, 0);
            acc0 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(bl0, ah[ks], acc0, 0, 0, 0);
            acc1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(bl1, ah[ks], acc1, 0, 0, 0);
            acc0 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(bh0, al[ks], acc0, 0, 0, 0);
            acc1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(bh1, al[ks], acc1, 0, 0, 0);
        }
        if constexpr (K <= 64) __builtin_amdgcn_s_setprio(0);
        screen(acc0, tile_row0(t), t * TR);
        screen(acc1, tile_row0(t) + kMfmaRows, t * TR + kMfmaRows);
        __syncthreads();
    }
    if (PILOT) {
        // ascending bitonic sort of the lane's 16 class minima, in registers
#pragma unroll
        for (int k = 2; k <= 16; k <<= 1) {
#pragma unroll
            for (int j = k >> 1; j > 0; j >>= 1) {
#pragma unroll
                for (int i = 0; i < 16; ++i) {
                    const int p = i ^ j;
                    if (p > i) {
                        const float x = cmin[i], y = cmin[p];
                        const bool up = (i & k) == 0;
                        cmin[i] = up ? fminf(x, y) : fmaxf(x, y);
                        cmin[p] = up ? fmaxf(x, y) : fminf(x, y);
                    }
                }
            }
        }
        // the other half-wavefront's sorted minima of the same voxel; the k-th
        // smallest of the two sorted lists a, b is the minimum over i of
        // max(a[i-1], b[k-1-i]) (an empty side counting as -inf)
        float pm[16];
#pragma unroll
        for (int r = 0; r < 16; ++r) pm[r] = __shfl_xor(cmin[r], 32, kWave);
        auto kth = [&](auto kc) {
            constexpr int k = decltype(kc)::value;
            float best = __builtin_inff();
#pragma unroll
            for (int i = 0; i <= k; ++i) {
                const float x = i > 0 ? cmin[i > 0 ? i - 1 : 0] : -__builtin_inff();
                const float y = i < k ? pm[i < k ? k - 1 - i : 0] : -__builtin_inff();
                best = fminf(best, fmaxf(x, y));
            }
            return best;
        };
        const float c16 = kth(std::integral_constant<int, kBankTopK>{});
        const float c8 = kth(std::integral_constant<int, kBankTopK / 2>{});
        if (half == 0 && v < P.V) {
            constexpr double m = contraction_rel_err<K>();
            // candidate test of threshold t: t - a + m E_t, E_t = 3a + 4 sqrt(a t) + t
            auto test_of = [&](float t, double a) {
                const double tp = fmax((double)t, 0.0);
                const double e_t = 3.0 * a + 4.0 * sqrt(a * tp) + tp;
                return (float)((double)t - a + m * e_t + 1e-6 * (a + fabs((double)t)));
            };
            const double a = P.aval[v];
            if (a < 0.0) {  // negative weights: no bound, every row a candidate
                P.tau[v] = P.tau1[v] = __builtin_inff();
                P.cthr[v] = P.cthr1[v] = __builtin_inff();
            } else if (a == a) {  // (NaN: invalid voxel, marked by the operand kernel)
                const float tau = (float)(a + (double)c16), tau1 = (float)(a + (double)c8);
                P.tau[v] = tau;
                P.cthr[v] = test_of(tau, a);
                P.tau1[v] = tau1;
                P.cthr1[v] = test_of(tau1, a);
            }
        }
    } else {
        const unsigned cnt = (lnext - loff) >> 3, other = __shfl_xor(cnt, 32, kWave);
        if (half == 0 && v < P.V && cth > -__builtin_inff()) {
            P.cnt[v] = (cnt > hcap || other > hcap) ? P.cap + 1 : (int)(cnt + other);
            P.cnt_hi[v] = (int)other;
        }
    }
}

// Up to 32 frames the kernel fits 128 VGPRs (4 wavefronts per SIMD, two
// blocks per CU); 40 and 48 frames need more registers and run at 3.
template <int K, bool PILOT>
__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(4))) void vpet_bank_mfma_kernel(BankArgs P) {
    bank_mfma_body<K, PILOT>(P);
}
template <int K, bool PILOT>
__global__ __launch_bounds__(512) void vpet_bank_mfma_wide_kernel(BankArgs P) {
    bank_mfma_body<K, PILOT>(P);
}

template <int K, bool PILOT>
void launch_mfma(dim3 grid, hipStream_t st, const BankArgs& Q) {
    if constexpr (K <= 64)
        hipLaunchKernelGGL((vpet_bank_mfma_kernel<K, PILOT>), grid, dim3(512), 0, st, Q);
    else
        hipLaunchKernelGGL((vpet_bank_mfma_wide_kernel<K, PILOT>), grid, dim3(512), 0, st, Q);
}

// ===========================================================================
// Learned proposal (not in the paper): an amortised importance sampler for the
// prior draws of Alg. 1.  A multilayer perceptron maps a voxel's observed TAC
// (features x_f = log1p(max(y_f, 0)), zero-padded to 32) through two ReLU
// layers of 256 to 72 outputs: 8 mixture logits, 8 x 4 means and 8 x 4 raw
// scales of a diagonal Gaussian mixture over z = log(theta) of the free
// parameters (K1, k2, k3, vB); log sd = LS0 + (LS1 - LS0) sigmoid(raw).  It is
// trained on simulated (theta, noisy TAC) pairs by minimising the mean
// negative log density of z, with bf16 matrix-core GEMMs (FP32 accumulation)
// and FP32 master weights updated by Adam.  Draws from the mixture are
// weighted by prior / proposal, so the ABC target is unchanged.
// ===========================================================================
constexpr int kMixC = 8, kMixD = 4;  // kMixD: the importance-weighted per-voxel path (irreversible 2TCM)
constexpr int kMixDMax = 5;          // a head over log(K1, k2, k3, k4, vB) for the reversible model
constexpr int kNetIn = 32, kNetH = 256, kNetOut = 96;
// outputs in use by a head over D parameters: 8 logits, 8 x D means, 8 x D raw scales
__host__ __device__ constexpr int net_out_used(int D) { return kMixC + 2 * kMixC * D; }
// theta slots of the D parameters of a head: (K1, k2, k3, vB) or (K1, k2, k3, k4, vB)
template <int D>
__device__ __forceinline__ int head_slot(int j) { return (D == 4 && j == 3) ? VPET_SLOT_VB : j; }
constexpr double kLS0 = -6.0, kLS1 = 2.0;
constexpr size_t kOffW1 = 0, kOffB1 = kOffW1 + (size_t)kNetIn * kNetH, kOffW2 = kOffB1 + kNetH,
                 kOffB2 = kOffW2 + (size_t)kNetH * kNetH, kOffW3 = kOffB2 + kNetH,
                 kOffB3 = kOffW3 + (size_t)kNetH * kNetOut, kNetParams = kOffB3 + kNetOut;
static_assert(kNetParams == VPET_PROPOSAL_NPARAM, "parameter blob layout");

// C = epilogue(op(A) op(B)): a(m, k) = A[m sam + k sak], b(k, n) = B[k sbk +
// n sbn], FP32 in memory, bf16 on the matrix cores, FP32 accumulation.
// Epilogue: + bias[n]; then ReLU (relu), or multiplication by (mask[m][n] > 0)
// (the ReLU derivative of the forward activation); accumulate adds to C.
struct GemmArgs {
    const float* A;
    long long sam, sak;
    const float* B;
    long long sbk, sbn;
    float* C;
    long long ldc;
    const float* bias;
    const float* mask;
    long long ldm;
    int M, N, K, relu, accumulate;
    // split K: block z sums k in [z kchunk, (z+1) kchunk) and, with part set,
    // stores its raw partial tile at part + z pstride ([M][N]); a second
    // kernel adds the partials in order and applies the epilogue
    int kchunk;
    float* part;
    long long pstride;
};

// Split of 8 fp32 values into bf16 hi = rn(x) and lo = rn(x - hi), packed.
__device__ __forceinline__ void split_bf16x8(const float (&x)[8], uint4& hi, uint4& lo) {
    uint32_t h[8], l[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) {
        h[e] = bf16_rn(x[e]);
        l[e] = bf16_rn(x[e] - __uint_as_float(h[e] << 16));
    }
    hi = make_uint4(h[0] | (h[1] << 16), h[2] | (h[3] << 16), h[4] | (h[5] << 16), h[6] | (h[7] << 16));
    lo = make_uint4(l[0] | (l[1] << 16), l[2] | (l[3] << 16), l[4] | (l[5] << 16), l[6] | (l[7] << 16));
}

// C = act(A B + bias) (or masked) with fp32 operands on BF16 matrix cores:
// each operand is split into bf16 hi + lo and the product is hi*hi + hi*lo +
// lo*hi (three MFMAs, FP32 accumulation), relative error about 3 * 2^-16 per
// term instead of 2^-7 for a plain bf16 product.
// Block = 4 wavefronts = a 64 x 64 tile of C (a 32 x 32 tile per wavefront).
// K advances in chunks of 32: the block stages the chunk's 64 x 32 slices of A
// and B into LDS, split into bf16 hi and lo once, with loads in which
// consecutive lanes read consecutive addresses along whichever of the
// operand's two strides is 1 (the transposed operands of the backward pass
// included); the wavefronts then read their MFMA fragments from LDS.  Two
// buffers: the loads of chunk c+1 are issued before chunk c is multiplied.
// The products and their order per 16-wide k step are those of one MFMA
// chain per output tile, so the result does not depend on the staging.
constexpr int kGemmKC = 32;                  // k per staged chunk
constexpr int kGemmRS = kGemmKC + 8;         // LDS row stride (bf16), padded against bank conflicts
__global__ __launch_bounds__(256) void vpet_gemm_bf16x3_kernel(GemmArgs G) {
    __shared__ __align__(16) uint16_t sm[2][4][64 * kGemmRS];  // [buffer][A hi, A lo, B hi, B lo][row][k]
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int bm0 = blockIdx.y * 64, bn0 = blockIdx.x * 64;
    const int m0 = bm0 + (wave >> 1) * 32, n0 = bn0 + (wave & 1) * 32;
    const int kbeg = blockIdx.z * G.kchunk, kend = min(G.K, kbeg + G.kchunk);
    // staging map: element e = tid + 256 q (q < 8) of a 64 x 32 slice, the
    // fast index along the operand's unit stride
    const bool a_kfast = G.sak == 1, b_kfast = G.sbk == 1;
    float av[8], bv[8];
    auto load = [&](int k0) {
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const int e = tid + 256 * q;
            {
                const int r = a_kfast ? (e >> 5) : (e & 63), k = a_kfast ? (e & 31) : (e >> 6);
                const int m = bm0 + r, kk = k0 + k;
                av[q] = (m < G.M && kk < kend) ? G.A[(long long)m * G.sam + (long long)kk * G.sak] : 0.0f;
            }
            {
                const int r = b_kfast ? (e >> 5) : (e & 63), k = b_kfast ? (e & 31) : (e >> 6);
                const int n = bn0 + r, kk = k0 + k;
                bv[q] = (n < G.N && kk < kend) ? G.B[(long long)kk * G.sbk + (long long)n * G.sbn] : 0.0f;
            }
        }
    };
    auto stash = [&](int buf) {
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const int e = tid + 256 * q;
            {
                const int r = a_kfast ? (e >> 5) : (e & 63), k = a_kfast ? (e & 31) : (e >> 6);
                const uint32_t h = bf16_rn(av[q]);
                sm[buf][0][r * kGemmRS + k] = (uint16_t)h;
                sm[buf][1][r * kGemmRS + k] = (uint16_t)bf16_rn(av[q] - __uint_as_float(h << 16));
            }
            {
                const int r = b_kfast ? (e >> 5) : (e & 63), k = b_kfast ? (e & 31) : (e >> 6);
                const uint32_t h = bf16_rn(bv[q]);
                sm[buf][2][r * kGemmRS + k] = (uint16_t)h;
                sm[buf][3][r * kGemmRS + k] = (uint16_t)bf16_rn(bv[q] - __uint_as_float(h << 16));
            }
        }
    };
    f32x16_t acc = {};
    const int nchunks = kend > kbeg ? (kend - kbeg + kGemmKC - 1) / kGemmKC : 0;
    if (nchunks > 0) {
        load(kbeg);
        stash(0);
        __syncthreads();
    }
    const int ar = (wave >> 1) * 32 + (lane & 31), br = (wave & 1) * 32 + (lane & 31), kk = 8 * (lane >> 5);
    for (int c = 0; c < nchunks; ++c) {
        const int buf = c & 1;
        if (c + 1 < nchunks) load(kbeg + (c + 1) * kGemmKC);  // in flight while this chunk is multiplied
#pragma unroll
        for (int ks = 0; ks < kGemmKC / 16; ++ks) {
            const int off = ks * 16 + kk;
            const bf16x8_t Ah = __builtin_bit_cast(bf16x8_t, *reinterpret_cast<const uint4*>(&sm[buf][0][ar * kGemmRS + off]));
            const bf16x8_t Al = __builtin_bit_cast(bf16x8_t, *reinterpret_cast<const uint4*>(&sm[buf][1][ar * kGemmRS + off]));
            const bf16x8_t Bh = __builtin_bit_cast(bf16x8_t, *reinterpret_cast<const uint4*>(&sm[buf][2][br * kGemmRS + off]));
            const bf16x8_t Bl = __builtin_bit_cast(bf16x8_t, *reinterpret_cast<const uint4*>(&sm[buf][3][br * kGemmRS + off]));
            acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(Al, Bh, acc, 0, 0, 0);
            acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(Ah, Bl, acc, 0, 0, 0);
            acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(Ah, Bh, acc, 0, 0, 0);
        }
        if (c + 1 < nchunks) {
            stash(buf ^ 1);  // the other buffer was last read before the previous barrier
            __syncthreads();
        }
    }
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        const int m = m0 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3), n = n0 + (lane & 31);
        if (m >= G.M || n >= G.N) continue;
        float v = acc[r];
        if (G.part) {
            G.part[blockIdx.z * G.pstride + (long long)m * G.N + n] = v;
            continue;
        }
        if (G.bias) v += G.bias[n];
        if (G.relu) v = fmaxf(v, 0.0f);
        if (G.mask && !(G.mask[(long long)m * G.ldm + n] > 0.0f)) v = 0.0f;
        float* cptr = G.C + (long long)m * G.ldc + n;
        *cptr = G.accumulate ? *cptr + v : v;
    }
}

// C = epilogue(sum over the S split-K partials, in order): bias, relu, mask.
__global__ __launch_bounds__(256) void vpet_gemm_reduce_kernel(GemmArgs G, int S) {
    const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (long long)G.M * G.N) return;
    const int m = (int)(e / G.N), n = (int)(e - (long long)m * G.N);
    float v = 0.0f;
    for (int z = 0; z < S; ++z) v += G.part[z * G.pstride + e];
    if (G.bias) v += G.bias[n];
    if (G.relu) v = fmaxf(v, 0.0f);
    if (G.mask && !(G.mask[(long long)m * G.ldm + n] > 0.0f)) v = 0.0f;
    float* c = G.C + (long long)m * G.ldc + n;
    *c = G.accumulate ? *c + v : v;
}

// db[n] = sum_m dY[m][n] (one block per column).
__global__ __launch_bounds__(256) void vpet_colsum_kernel(const float* dY, long long ld, int M, float* out) {
    const int n = blockIdx.x;
    double s = 0.0;
    for (int m = threadIdx.x; m < M; m += blockDim.x) s += (double)dY[(long long)m * ld + n];
    __shared__ double part[4];
    s = wave_sum(s);
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) out[n] = (float)(part[0] + part[1] + part[2] + part[3]);
}

// Mean negative log density of z[b][D] under the mixture of O[b][96] (a head
// over D parameters) and its gradient dO (already divided by the batch size);
// loss_acc += mean.
template <int D>
__global__ __launch_bounds__(256) void vpet_mix_loss_kernel(const float* O, const float* Z, int Bn, float* dO,
                                                            float* loss_acc) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    double nll = 0.0;
    if (b < Bn) {
        const float* o = O + (size_t)b * kNetOut;
        float* d = dO + (size_t)b * kNetOut;
        double lg[kMixC], comp[kMixC], mx = -1e300;
#pragma unroll
        for (int c = 0; c < kMixC; ++c) mx = fmax(mx, (double)o[c]);
        double se = 0.0;
#pragma unroll
        for (int c = 0; c < kMixC; ++c) se += exp((double)o[c] - mx);
        const double lse_l = mx + log(se);
        double cmx = -1e300;
#pragma unroll
        for (int c = 0; c < kMixC; ++c) {
            lg[c] = (double)o[c] - lse_l;  // log pi_c
            double q = lg[c];
#pragma unroll
            for (int j = 0; j < D; ++j) {
                const double sg = 1.0 / (1.0 + exp(-(double)o[kMixC + kMixC * D + c * D + j]));
                const double lsd = kLS0 + (kLS1 - kLS0) * sg;
                const double t = ((double)Z[b * D + j] - (double)o[kMixC + c * D + j]) * exp(-lsd);
                q += -0.5 * t * t - lsd - 0.9189385332046727;  // 0.5 log(2 pi)
            }
            comp[c] = q;
            cmx = fmax(cmx, q);
        }
        double sc = 0.0;
#pragma unroll
        for (int c = 0; c < kMixC; ++c) sc += exp(comp[c] - cmx);
        const double lse = cmx + log(sc);
        nll = -lse;
        const double rB = 1.0 / (double)Bn;
#pragma unroll
        for (int c = 0; c < kMixC; ++c) {
            const double r = exp(comp[c] - lse);
            d[c] = (float)((exp(lg[c]) - r) * rB);
#pragma unroll
            for (int j = 0; j < D; ++j) {
                const double sg = 1.0 / (1.0 + exp(-(double)o[kMixC + kMixC * D + c * D + j]));
                const double lsd = kLS0 + (kLS1 - kLS0) * sg;
                const double isd = exp(-lsd);
                const double t = ((double)Z[b * D + j] - (double)o[kMixC + c * D + j]) * isd;
                d[kMixC + c * D + j] = (float)(-r * t * isd * rB);
                d[kMixC + kMixC * D + c * D + j] = (float)(r * (1.0 - t * t) * (kLS1 - kLS0) * sg * (1.0 - sg) * rB);
            }
        }
        for (int q = net_out_used(D); q < kNetOut; ++q) d[q] = 0.0f;
    }
    __shared__ double part[4];
    double s = wave_sum(nll);
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) atomicAdd(loss_acc, (float)((part[0] + part[1] + part[2] + part[3]) / (double)Bn));
}

// Adam (Kingma and Ba) on the FP32 master weights; c1, c2 are the bias
// corrections 1 / (1 - beta^t).
__global__ __launch_bounds__(256) void vpet_adam_kernel(float* p, const float* g, float* m, float* v, long long n,
                                                        float lr, float c1, float c2) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = 0.9f * m[i] + 0.1f * gi, vi = 0.999f * v[i] + 0.001f * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi * c1) / (sqrtf(vi * c2) + 1e-8f);
}

// He-normal weights (sd sqrt(2 / fan_in); the output layer sqrt(1 / fan_in)),
// zero biases; normals from Philox stream 5 by Box-Muller.
__global__ __launch_bounds__(256) void vpet_net_init_kernel(float* p, uint32_t key0, uint32_t key1) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (long long)kNetParams) return;
    double sd = 0.0;
    if (i < (long long)kOffB1) sd = sqrt(2.0 / kNetIn);
    else if (i >= (long long)kOffW2 && i < (long long)kOffB2) sd = sqrt(2.0 / kNetH);
    else if (i >= (long long)kOffW3 && i < (long long)kOffB3) sd = sqrt(1.0 / kNetH);
    uint32_t w[4];
    philox10((uint32_t)i, 0u, 5u, 0u, key0, key1, w);
    const double ua = ((double)(w[0] >> 8) + 1.0) * 0x1p-24, ub = (double)(w[1] >> 8) * 0x1p-24;
    p[i] = (float)(sd * sqrt(-2.0 * log(ua)) * cos(2.0 * M_PI * ub));
}

// Network inputs X[b][32] = log1p(max(y, 0)) (zero padding) of observed TACs.
__global__ __launch_bounds__(256) void vpet_net_features_kernel(const float* tacs, long long n, int F, float* X) {
    const long long b = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= n) return;
    for (int f = 0; f < kNetIn; ++f)
        X[b * kNetIn + f] = f < F ? (float)log1p(fmax((double)tacs[b * F + f], 0.0)) : 0.0f;
}

// Training batch: bank row of sample j of epoch e is (j * mul + add) mod n_bank
// (mul coprime with n_bank); the TAC gets fresh Gaussian noise
// sd_f = sqrt(fac_f max(x_f, 0)) (fac_f = level e^{lambda tmid_f} / dt_f,
// normals from Philox stream 4, counter (row, e, 4, f/4)); inputs as above and
// targets z = log(max(theta, 1e-6)) of the head's D parameters.
template <int D>
__global__ __launch_bounds__(256) void vpet_net_batch_kernel(const float* bank_theta, const double* bank_x, int ld,
                                                             long long n_bank, int F, const double* fac,
                                                             unsigned long long j0, unsigned long long mul,
                                                             unsigned long long add, uint32_t epoch, int Bn,
                                                             uint32_t key0, uint32_t key1, float* X, float* Z) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= Bn) return;
    const unsigned long long row = ((j0 + (unsigned long long)b) % (unsigned long long)n_bank * mul + add) %
                                   (unsigned long long)n_bank;
    const float* t = bank_theta + row * VPET_PSTRIDE;
#pragma unroll
    for (int j = 0; j < D; ++j) Z[b * D + j] = (float)log(fmax((double)t[head_slot<D>(j)], 1e-6));
    const double* x = bank_x + row * (size_t)ld;
    for (int f0 = 0; f0 < kNetIn; f0 += 4) {
        uint32_t w[4];
        philox10((uint32_t)row, epoch, 4u, (uint32_t)(f0 >> 2), key0, key1, w);
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            const double ua = ((double)(w[2 * q] >> 8) + 1.0) * 0x1p-24, ub = (double)(w[2 * q + 1] >> 8) * 0x1p-24;
            const double r = sqrt(-2.0 * log(ua));
            double sn, cs;
            sincos(2.0 * M_PI * ub, &sn, &cs);
#pragma unroll
            for (int e = 0; e < 2; ++e) {
                const int f = f0 + 2 * q + e;
                float v = 0.0f;
                if (f < F) {
                    const double xf = x[f];
                    const double y = xf + sqrt(fac[f] * fmax(xf, 0.0)) * (e ? sn : cs) * r;
                    v = (float)log1p(fmax(y, 0.0));
                }
                X[(size_t)b * kNetIn + f] = v;
            }
        }
    }
}

// Per-voxel mixture in FP64 (the proposal of voxel row), kept in LDS.
struct MixTab {
    double cum[kMixC], logpi[kMixC];
    double mu[kMixC * kMixD], sd[kMixC * kMixD], logsd[kMixC * kMixD];
    double share, log_share, log_rest, logvol;
    float lo[kMixD], hi[kMixD];  // fp32 prior box of the drawn parameters
};

// Mixture of one voxel's outputs o[72]: weights softmax(logits), log sd =
// LS0 + (LS1 - LS0) sigmoid(raw) + logscale; cum[c] = a + (1 - a) (pi_0 + ...
// + pi_c), the component thresholds of u0 above the defensive share a.
__device__ void mix_table(const float* o, MixTab& t, double share, double logscale, double logvol, const float* lo,
                          const float* hi) {
    double mx = -1e300;
    for (int c = 0; c < kMixC; ++c) mx = fmax(mx, (double)o[c]);
    double se = 0.0;
    for (int c = 0; c < kMixC; ++c) se += exp((double)o[c] - mx);
    const double lse = mx + log(se);
    double run = 0.0;
    for (int c = 0; c < kMixC; ++c) {
        t.logpi[c] = (double)o[c] - lse;
        run += exp(t.logpi[c]);
        t.cum[c] = share + (1.0 - share) * run;
        for (int j = 0; j < kMixD; ++j) {
            const int q = c * kMixD + j;
            t.mu[q] = (double)o[kMixC + q];
            t.logsd[q] = kLS0 + (kLS1 - kLS0) / (1.0 + exp(-(double)o[kMixC + kMixC * kMixD + q]));
            if (logscale != 0.0) t.logsd[q] += logscale;
            t.sd[q] = exp(t.logsd[q]);
        }
    }
    for (int j = 0; j < kMixD; ++j) {
        t.lo[j] = lo[j];
        t.hi[j] = hi[j];
    }
    t.share = share;
    t.log_share = log(share);
    t.log_rest = log1p(-share);
    t.logvol = logvol;
}

// FP64 log and exp for the proposal draws, from their series (within 1 ulp
// of the library functions, at about a third of their instructions):
//   log x = e ln 2 + 2 atanh(s), x = m 2^e, m in [1/sqrt 2, sqrt 2),
//           s = (m - 1)/(m + 1), atanh by its odd series to s^23 (|s| < 0.172);
//   exp z = 2^k e^r, k = rint(z log2 e), r = z - k ln 2 (|r| <= 0.347), e^r by
//           its Taylor series to r^13;
// ln 2 is split into hi = ln 2 rounded to float (k hi exact) and lo = the rest.
// log_pos needs a finite x > 0.
constexpr double kLn2Hi = 0.693147182464599609375, kLn2Lo = -1.9046542999577693e-09;

__device__ __forceinline__ double log_pos(double x) {
    int e;
    double m = frexp(x, &e);
    if (m < 0.70710678118654752) {
        m *= 2.0;
        e -= 1;
    }
    const double s = (m - 1.0) / (m + 1.0), s2 = s * s;
    double p = 1.0 / 23.0;
    p = fma(p, s2, 1.0 / 21.0);
    p = fma(p, s2, 1.0 / 19.0);
    p = fma(p, s2, 1.0 / 17.0);
    p = fma(p, s2, 1.0 / 15.0);
    p = fma(p, s2, 1.0 / 13.0);
    p = fma(p, s2, 1.0 / 11.0);
    p = fma(p, s2, 1.0 / 9.0);
    p = fma(p, s2, 1.0 / 7.0);
    p = fma(p, s2, 1.0 / 5.0);
    p = fma(p, s2, 1.0 / 3.0);
    const double lm = fma(2.0 * s, s2 * p, 2.0 * s);
    const double de = (double)e;
    return fma(de, kLn2Hi, fma(de, kLn2Lo, lm));
}

__device__ __forceinline__ double exp_series(double z) {
    const double k = rint(z * 1.4426950408889634);
    double r = fma(-k, kLn2Hi, z);
    r = fma(-k, kLn2Lo, r);
    double p = 1.0 / 6227020800.0;  // 1/13!
    p = fma(p, r, 1.0 / 479001600.0);
    p = fma(p, r, 1.0 / 39916800.0);
    p = fma(p, r, 1.0 / 3628800.0);
    p = fma(p, r, 1.0 / 362880.0);
    p = fma(p, r, 1.0 / 40320.0);
    p = fma(p, r, 1.0 / 5040.0);
    p = fma(p, r, 1.0 / 720.0);
    p = fma(p, r, 1.0 / 120.0);
    p = fma(p, r, 1.0 / 24.0);
    p = fma(p, r, 1.0 / 6.0);
    p = fma(p, r, 0.5);
    p = fma(p, r, 1.0);
    p = fma(p, r, 1.0);
    return ldexp(p, (int)k);
}

// Proposal draw i of voxel v: one Philox block (stream 2), u0 from the low
// bytes of words 0-2, u_j = (w_j >> 8) 2^-24.  u0 below the defensive share
// draws theta uniformly from the box (z = log theta); otherwise a component
// by inverse CDF and Box-Muller normals give z, theta = fp32(exp(z)).  Draw
// order of the irreversible 2TCM (K1, k2, k3, vB).  False outside the box.
// With WANT_Z false, z is not formed for prior draws (the screening pass
// needs theta only).
template <bool WANT_Z>
__device__ __forceinline__ bool proposal_draw(const MixTab& t, uint32_t key0, uint32_t key1, uint32_t v, uint32_t i,
                                              float th[kMaxParams], double z[kMixD]) {
    const float* lo = t.lo;
    const float* hi = t.hi;
    uint32_t w[4];
    philox10(i, v, 2u, 0u, key0, key1, w);
    const double u0 = (double)((w[0] & 255u) | (w[1] & 255u) << 8 | (w[2] & 255u) << 16) * 0x1p-24;
    double u[kMixD];
#pragma unroll
    for (int j = 0; j < kMixD; ++j) u[j] = (double)(w[j] >> 8) * 0x1p-24;
#pragma unroll
    for (int j = kMixD; j < kMaxParams; ++j) th[j] = 0.0f;
    if (u0 < t.share) {
#pragma unroll
        for (int j = 0; j < kMixD; ++j) {
            th[j] = (float)((double)lo[j] + u[j] * ((double)hi[j] - (double)lo[j]));
            if (WANT_Z) z[j] = log((double)th[j]);
        }
        return true;
    }
    int c = 0;
#pragma unroll
    for (int q = 0; q < kMixC - 1; ++q) c += (t.cum[q] <= u0) ? 1 : 0;
    double nrm[kMixD];
#pragma unroll
    for (int q = 0; q < 2; ++q) {
        const double r = sqrt(-2.0 * log_pos(u[2 * q] + 0x1p-24));
        double sn, cs;
        sincospi(2.0 * u[2 * q + 1], &sn, &cs);  // angle 2 pi u, reduced exactly
        nrm[2 * q] = r * cs;
        nrm[2 * q + 1] = r * sn;
    }
    bool ok = true;
#pragma unroll
    for (int j = 0; j < kMixD; ++j) {
        const double zj = t.mu[c * kMixD + j] + t.sd[c * kMixD + j] * nrm[j];
        if (WANT_Z) z[j] = zj;
        th[j] = (float)exp_series(zj);
        ok = ok && th[j] >= lo[j] && th[j] <= hi[j];
    }
    return ok;
}

// The screening pass's draw as an out-of-line call: its transcendental
// functions' FP64 constants are then formed inside the call instead of being
// hoisted (and kept live, or spilled) across the whole simulation loop.
struct ThetaDraw {
    float th[kMixD];
    int ok;
};

__device__ __attribute__((noinline)) ThetaDraw proposal_theta(const MixTab* t, uint32_t key0, uint32_t key1,
                                                              uint32_t v, uint32_t i) {
    ThetaDraw r;
    float th[kMaxParams];
    double z[kMixD];
    r.ok = proposal_draw<false>(*t, key0, key1, v, i, th, z) ? 1 : 0;
#pragma unroll
    for (int j = 0; j < kMixD; ++j) r.th[j] = th[j];
    return r;
}

// log w = -log(a + (1 - a) e^L), L = log q(z) - sum_j z_j + logvol the log
// ratio proposal / prior in theta space (sum_j z_j: the Jacobian of exp);
// L = -inf where some theta_j = 0.  With a = 0 simply -L.
__device__ __forceinline__ double proposal_log_weight(const MixTab& t, const double z[kMixD]) {
    bool fin = true;
#pragma unroll
    for (int j = 0; j < kMixD; ++j) fin = fin && isfinite(z[j]);
    if (!fin) return -t.log_share;
    double comp[kMixC], mx = -1e300;
#pragma unroll
    for (int c = 0; c < kMixC; ++c) {
        double q = t.logpi[c];
#pragma unroll
        for (int j = 0; j < kMixD; ++j) {
            const double u = (z[j] - t.mu[c * kMixD + j]) / t.sd[c * kMixD + j];
            q += -0.5 * u * u - t.logsd[c * kMixD + j] - 0.9189385332046727;
        }
        comp[c] = q;
        mx = fmax(mx, q);
    }
    double s = 0.0;
#pragma unroll
    for (int c = 0; c < kMixC; ++c) s += exp(comp[c] - mx);
    double zs = 0.0;
#pragma unroll
    for (int j = 0; j < kMixD; ++j) zs += z[j];
    const double L = (mx + log(s)) - zs + t.logvol;
    if (t.share == 0.0) return -L;
    const double x = t.log_share, y = t.log_rest + L;  // -logaddexp(x, y)
    const double m = fmax(x, y);
    return -(m + log1p(exp(-fabs(x - y))));
}

// Keys of one tile of proposal draws (invalid draws never enter the top n).
template <int U, bool L1>
__device__ __forceinline__ void tile_keys_is(const InferArgs& P, const MixTab& mix, uint32_t v, uint32_t i0,
                                             const double2* yw, uint64_t (&key)[U]) {
    DrawState<1, U> s;
    uint32_t idx[U];
    bool ok[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const uint32_t i = i0 + (uint32_t)(u * kWave + lane_id());
        idx[u] = i < P.n_draws ? i : P.n_draws - 1;
        float th[kMaxParams];
        const ThetaDraw d = proposal_theta(&mix, P.key0, P.key1, v, idx[u]);
#pragma unroll
        for (int j = 0; j < kMixD; ++j) th[j] = d.th[j];
#pragma unroll
        for (int j = kMixD; j < kMaxParams; ++j) th[j] = 0.0f;
        ok[u] = d.ok && i < P.n_draws;
        if (!ok[u]) {  // a harmless in-box stand-in keeps the lane's recursion finite
            th[0] = mix.hi[0];
            th[1] = mix.hi[1];
            th[2] = mix.lo[2];
            th[3] = mix.lo[3];
        }
        setup<KIND_IRR, 1, U>(th, P.h, P.C0, s, u);
    }
    DistSink<U, L1> sink;
    sink.yw = yw;
#pragma unroll
    for (int u = 0; u < U; ++u) sink.d[u] = 0.0;
    simulate_draws<KIND_IRR, U>(P.tab, P.F, P.k0, s, sink);
#pragma unroll
    for (int u = 0; u < U; ++u) {
        float fd = (float)sink.d[u];
        if (!(fd == fd)) fd = __builtin_inff();
        key[u] = ok[u] ? (((uint64_t)__float_as_uint(fd) << 32) | idx[u]) : kNoKey;
    }
}

__device__ double block_max(double v, double* red, int nw) {
    v = wave_max(v);
    if (lane_id() == 0) red[(threadIdx.x >> 6) * kRedStride] = v;
    __syncthreads();
    double m = -__builtin_inf();
    for (int w = 0; w < nw; ++w) m = fmax(m, red[w * kRedStride]);
    __syncthreads();
    return m;
}

// Importance-weighted ABC of one voxel per block (irreversible 2TCM): n_draws
// proposal draws from the voxel's mixture, the n closest valid ones accepted,
// moments weighted by prior / proposal (FP64, max-shifted), and the effective
// sample size (sum w)^2 / sum w^2.
// (At most 128 VGPRs for four waves per SIMD: the few spills this costs sit
// in the accepted-draw epilogue, not in the screening loop.)
template <bool L1>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) void vpet_infer_is_kernel(InferArgs P) {
    extern __shared__ __align__(16) unsigned char lds[];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const long long row = blockIdx.x;
    if (row >= P.V) return;
    const int F = P.F;
    const uint32_t vg = (uint32_t)(P.vbase + (unsigned long long)row);
    double2* yw = reinterpret_cast<double2*>(lds);
    const int yw_bytes = (16 * F + 15) & ~15;
    uint64_t* keys_all = reinterpret_cast<uint64_t*>(lds + yw_bytes);
    double* red = reinterpret_cast<double*>(keys_all + (size_t)P.wpv * P.cap);
    int* flag = reinterpret_cast<int*>(red + kRedStride * kMaxWpv);
    MixTab* mix = reinterpret_cast<MixTab*>(reinterpret_cast<unsigned char*>(flag) + 16);
    const int n = (int)P.n_acc;
    if (wave == 0) {
        const float* y = P.tacs + (size_t)row * F;
        const cdp FR = (cdp)P.tab.fr;
        const cip NF = (cip)P.tab.nf;
        float ymax = -__builtin_inff();
        int bad = 0;
        for (int f = lane; f < F; f += kWave) {
            const float yy = y[f];
            bad |= !isfinite(yy);
            ymax = fmaxf(ymax, yy);
            if (P.weights) {  // caller weights must be finite and >= 0
                const float wv = P.weights[(size_t)row * F + f];
                bad |= !(wv >= 0.0f) || !isfinite(wv);
            }
        }
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
            ymax = fmaxf(ymax, __shfl_xor(ymax, off, kWave));
            bad |= __shfl_xor(bad, off, kWave);
        }
        const bool valid = !bad && ymax > 0.0f;
        const double den_floor = P.floor_frac * (double)ymax;
        for (int f = lane; f < F; f += kWave) {
            const double nfd = (double)NF[f];
            const double yy = (double)y[f];
            double w;
            if (P.weights) {
                w = (double)P.weights[(size_t)row * F + f];
            } else {
                const double den = yy > den_floor ? yy : den_floor;
                w = FR[4 * f + 3] / den;
            }
            const double sw = sqrt(w);
            yw[f] = P.l1 ? make_double2(nfd * yy, sw / nfd) : make_double2(sw * yy, sw / nfd);
        }
        if (lane == 0) {
            *flag = valid ? 1 : 0;
            mix_table(P.prop + (size_t)row * kNetOut, *mix, P.prop_share, P.prop_logscale, P.prop_logvol, P.plo,
                      P.phi);
        }
    }
    __syncthreads();
    if (*flag == 0) {
        if (wave == 0) {
            const float qnan = __builtin_nanf("");
            for (int j = lane; j < 16; j += kWave) P.out_mom[(size_t)row * 16 + j] = qnan;
            if (lane == 0) {
                P.out_prob[row] = qnan;
                if (P.out_ess) P.out_ess[row] = qnan;
                if (P.out_thr) P.out_thr[row] = qnan;
            }
            if (P.out_idx)
                for (int j = lane; j < n; j += kWave) P.out_idx[(size_t)row * n + j] = -1;
            if (P.out_dist)
                for (int j = lane; j < n; j += kWave) P.out_dist[(size_t)row * n + j] = qnan;
        }
        return;
    }
    TopN top;
    top.keys = keys_all + (size_t)wave * P.cap;
    top.n = n;
    top.cap = P.cap;
    top.nbuf = 0;
    top.tau = kNoKey;
    for (int j = lane; j < P.cap; j += kWave) top.keys[j] = kNoKey;
    wave_lds_sync();
    constexpr int kU = kUmax;
    constexpr int kTile = kWave * kU;
    const uint32_t ntiles = (P.n_draws + kTile - 1) / kTile;
    for (uint32_t t = (uint32_t)wave; t < ntiles; t += (uint32_t)P.wpv) {
        uint64_t key[kU];
        tile_keys_is<kU, L1>(P, *mix, vg, t * kTile, yw, key);
        top.insert(key);
    }
    top.merge();
    __syncthreads();
    if (P.wpv > 1) block_topn_sort(keys_all, P.wpv, P.cap, n);
    const uint64_t* acc = keys_all;
    if (P.out_idx)
        for (int j = tid; j < n; j += blockDim.x)
            P.out_idx[(size_t)row * n + j] = acc[j] == kNoKey ? -1 : (int)(uint32_t)acc[j];
    if (P.out_dist)
        for (int j = tid; j < n; j += blockDim.x) P.out_dist[(size_t)row * n + j] = __uint_as_float((uint32_t)(acc[j] >> 32));
    if (P.out_thr && tid == 0) P.out_thr[row] = __uint_as_float((uint32_t)(acc[n - 1] >> 32));

    // weights of the accepted draws: max, then sums, then the spread
    const int nw = blockDim.x >> 6;
    const float h_v = P.below ? P.below[row] : __builtin_inff();
    auto accepted = [&](int j, float th[kMaxParams], double& lw) {
        if (acc[j] == kNoKey) return false;
        if (!(__uint_as_float((uint32_t)(acc[j] >> 32)) <= h_v)) return false;  // given threshold
        double z[kMixD];
        proposal_draw<true>(*mix, P.key0, P.key1, vg, (uint32_t)acc[j], th, z);
        lw = proposal_log_weight(*mix, z);
        return true;
    };
    double lmax = -__builtin_inf();
    for (int j = tid; j < n; j += blockDim.x) {
        float th[kMaxParams];
        double lw;
        if (accepted(j, th, lw)) lmax = fmax(lmax, lw);
    }
    lmax = block_max(lmax, red, nw);
    double s1[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) s1[q] = 0.0;  // sum w val[0..5], sum w, sum w^2
    for (int j = tid; j < n; j += blockDim.x) {
        float th[kMaxParams];
        double lw;
        if (!accepted(j, th, lw)) continue;
        const double w = exp(lw - lmax);
        double val[6];
        slot_values(KIND_IRR, th, val);
#pragma unroll
        for (int q = 0; q < 6; ++q) s1[q] = fma(w, val[q], s1[q]);
        s1[6] += w;
        s1[7] = fma(w, w, s1[7]);
    }
    block_sum<8>(s1, red, nw);
    const double sw = s1[6];
    double mean[6], s2[6];
#pragma unroll
    for (int q = 0; q < 6; ++q) {
        mean[q] = s1[q] / sw;
        s2[q] = 0.0;
    }
    for (int j = tid; j < n; j += blockDim.x) {
        float th[kMaxParams];
        double lw;
        if (!accepted(j, th, lw)) continue;
        const double w = exp(lw - lmax);
        double val[6];
        slot_values(KIND_IRR, th, val);
#pragma unroll
        for (int q = 0; q < 6; ++q) {
            const double dv = val[q] - mean[q];
            s2[q] = fma(w * dv, dv, s2[q]);
        }
    }
    block_sum<6>(s2, red, nw);
    if (tid < 16) {
        const int q = tid >> 1;
        float outv = __builtin_nanf("");
        if (q < 6 && slot_used(KIND_IRR, q) && sw > 0.0) outv = (tid & 1) == 0 ? (float)mean[q] : (float)(s2[q] / sw);
        P.out_mom[(size_t)row * 16 + tid] = outv;
    }
    if (tid == 0) {
        P.out_prob[row] = sw > 0.0 ? 1.0f : __builtin_nanf("");
        if (P.out_ess) P.out_ess[row] = sw > 0.0 ? (float)(sw * sw / s1[7]) : __builtin_nanf("");
    }
}

// ===========================================================================
// Learned-proposal bank (not in the paper): the shared bank of Alg. 1 drawn
// from a proposal fitted to a group of voxels instead of the prior.  Voxels
// are ordered by the cell of their network posterior (a serpentine walk over
// a grid on the prior box, so that consecutive cells are neighbours), cut into
// groups of S consecutive voxels, and each group gets one diagonal Gaussian in
// z = log(theta), moment-matched to its members' mixtures, mixed with the
// prior (defensive share a).  Every bank row carries the importance weight
// prior / proposal, so each voxel's ABC target is unchanged.
// ===========================================================================
constexpr int kLbMaxDims = 5;
constexpr int kLbBlock = 1024;        // voxels per histogram / scatter block
constexpr int kLbMaxCells = 4096;     // bins^dims
constexpr int kLbVox = kMfmaVox;      // groups hold whole tiles of the scans

struct LbArgs {
    const float* prop;     // [V][96] network outputs
    const float* tacs;     // [V][F]
    const float* weights;  // [V][F] caller weights or nullptr
    long long V;
    int F, D, bins, ncell, nb;
    float clo[kLbMaxDims], cwid[kLbMaxDims];  // prior box of the head's parameters (cells)
    unsigned* key;         // [V] cell along the serpentine walk; ncell for an invalid voxel
    double* zmom;          // [V][2 D] mixture mean and second moment of z
    int* hist;             // [nb][ncell + 1] block counts, then output offsets
    int* perm;             // [V] voxel at each position of the grouped order
    long long S;           // voxels per group
    int* out_group;        // [V] group of each voxel (optional)
    float* ys;             // [V][F] observed curves in the grouped order
    float* ws;             // [V][F] caller weights in the grouped order (with weights)
};

struct LbGroup {
    float mu[kLbMaxDims], sd[kLbMaxDims];
    int cnt;  // valid members; 0: the group's rows are prior draws
};

// Per voxel: validity (as in the bank form), the mixture moments of z and the
// cell key.  Mixture mean m_j = sum_c pi_c mu_cj and second moment
// s_j = sum_c pi_c (sd_cj^2 + mu_cj^2); cell coordinate j is
// floor(bins (exp(m_j) - lo_j) / (hi_j - lo_j)) clamped to [0, bins - 1]; the
// key walks the grid in serpentine order: coordinate j runs backwards when
// the key of the coordinates before it is odd.
// The voxel's whole network-output row and its TAC row are loaded before use
// (independent loads in flight together: the kernel is bound by their
// latency); D is a template parameter so that every index into them is a
// constant.
template <int D>
__device__ __forceinline__ void lb_summary(const LbArgs& A, long long v) {
    const float* yr = A.tacs + (size_t)v * A.F;
    bool bad = false;
    float ymax = -__builtin_inff();
    for (int f0 = 0; f0 < A.F; f0 += 16) {  // sixteen frames' loads in flight at a time
        float y[16];
#pragma unroll
        for (int i = 0; i < 16; ++i) y[i] = f0 + i < A.F ? yr[f0 + i] : 0.0f;
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            if (f0 + i >= A.F) break;
            bad = bad || !isfinite(y[i]);
            ymax = fmaxf(ymax, y[i]);
        }
    }
    float o[kNetOut];
    const float4* o4 = reinterpret_cast<const float4*>(A.prop + (size_t)v * kNetOut);
#pragma unroll
    for (int i = 0; i < kNetOut / 4; ++i) {
        const float4 q = o4[i];
        o[4 * i] = q.x;
        o[4 * i + 1] = q.y;
        o[4 * i + 2] = q.z;
        o[4 * i + 3] = q.w;
    }
    if (A.weights) {
        for (int f = 0; f < A.F; ++f) {
            const float w = A.weights[(size_t)v * A.F + f];
            bad = bad || !(w >= 0.0f) || !isfinite(w);
        }
    }
    double mx = -1e300;
#pragma unroll
    for (int c = 0; c < kMixC; ++c) mx = fmax(mx, (double)o[c]);
    double pi[kMixC], se = 0.0;
#pragma unroll
    for (int c = 0; c < kMixC; ++c) {
        pi[c] = exp((double)o[c] - mx);
        se += pi[c];
    }
    unsigned k = 0u;
    double* zm = A.zmom + (size_t)v * 2 * D;
#pragma unroll
    for (int j = 0; j < D; ++j) {
        double m = 0.0, s2 = 0.0;
#pragma unroll
        for (int c = 0; c < kMixC; ++c) {
            const double mu = (double)o[kMixC + c * D + j];
            const double lsd = kLS0 + (kLS1 - kLS0) / (1.0 + exp(-(double)o[kMixC + kMixC * D + c * D + j]));
            const double p = pi[c] / se;
            m = fma(p, mu, m);
            s2 = fma(p, exp(2.0 * lsd) + mu * mu, s2);
        }
        zm[2 * j] = m;
        zm[2 * j + 1] = s2;
        bad = bad || !isfinite(m) || !isfinite(s2);
        const double t = floor((double)A.bins * (exp(m) - (double)A.clo[j]) / (double)A.cwid[j]);
        int b = (t >= (double)A.bins) ? A.bins - 1 : (t >= 0.0 ? (int)t : 0);
        if (k & 1u) b = A.bins - 1 - b;
        k = k * (unsigned)A.bins + (unsigned)b;
    }
    A.key[v] = (bad || !(ymax > 0.0f)) ? (unsigned)A.ncell : k;
}

__global__ __launch_bounds__(256) void vpet_lb_summary_kernel(LbArgs A) {
    const long long v = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= A.V) return;
    if (A.D == 4)
        lb_summary<4>(A, v);
    else
        lb_summary<5>(A, v);
}

// Counts of each key (ncell + 1 values) in each block of kLbBlock voxels.
__global__ __launch_bounds__(256) void vpet_lb_hist_kernel(LbArgs A) {
    __shared__ int h[kLbMaxCells + 1];
    for (int c = threadIdx.x; c <= A.ncell; c += blockDim.x) h[c] = 0;
    __syncthreads();
    const long long v0 = (long long)blockIdx.x * kLbBlock;
    for (int i = threadIdx.x; i < kLbBlock; i += blockDim.x)
        if (v0 + i < A.V) atomicAdd(&h[A.key[v0 + i]], 1);
    __syncthreads();
    for (int c = threadIdx.x; c <= A.ncell; c += blockDim.x) A.hist[(size_t)blockIdx.x * (A.ncell + 1) + c] = h[c];
}

// Block counts -> first output position of each (block, key): keys in order,
// blocks in order within a key.  Pass 1 (a thread per key): each key's
// running count over the blocks and its total; pass 2 (one block): the
// exclusive scan of the totals, which the scatter adds.
__global__ __launch_bounds__(256) void vpet_lb_columns_kernel(LbArgs A, int* tot) {
    const int nc = A.ncell + 1;
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= nc) return;
    int run = 0;
    for (int b0 = 0; b0 < A.nb; b0 += 8) {  // eight blocks' counts loaded together
        int t[8];
#pragma unroll
        for (int i = 0; i < 8; ++i) t[i] = b0 + i < A.nb ? A.hist[(size_t)(b0 + i) * nc + c] : 0;
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            if (b0 + i >= A.nb) break;
            A.hist[(size_t)(b0 + i) * nc + c] = run;
            run += t[i];
        }
    }
    tot[c] = run;
}

__global__ __launch_bounds__(1024) void vpet_lb_cellbase_kernel(LbArgs A, int* tot) {
    __shared__ int part[1024];
    const int nc = A.ncell + 1, t = threadIdx.x;
    const int per = (nc + 1023) / 1024, c0 = t * per, c1 = min(nc, c0 + per);
    int s = 0;
    for (int c = c0; c < c1; ++c) s += tot[c];
    part[t] = s;
    __syncthreads();
    if (t == 0) {  // exclusive scan of the 1024 partial sums, in order
        int run = 0;
        for (int i = 0; i < 1024; ++i) {
            const int v = part[i];
            part[i] = run;
            run += v;
        }
    }
    __syncthreads();
    int run = part[t];
    for (int c = c0; c < c1; ++c) {
        const int v = tot[c];
        tot[c] = run;
        run += v;
    }
}

// Stable placement: one wavefront per block of kLbBlock voxels walks them in
// index order, 64 at a time; a voxel's position is its key's next free slot
// plus the number of earlier lanes of the same round with the same key.
__global__ __launch_bounds__(64) void vpet_lb_scatter_kernel(LbArgs A, const int* cellbase) {
    __shared__ int next[kLbMaxCells + 1];
    const int nc = A.ncell + 1, lane = threadIdx.x;
    for (int c = lane; c < nc; c += kWave) next[c] = cellbase[c] + A.hist[(size_t)blockIdx.x * nc + c];
    wave_lds_sync();
    const long long v0 = (long long)blockIdx.x * kLbBlock;
    for (int r = 0; r < kLbBlock / kWave; ++r) {
        const long long v = v0 + r * kWave + lane;
        const unsigned k = v < A.V ? A.key[v] : 0xFFFFFFFFu;
        int before = 0, after = 0;
        for (int q = 0; q < kWave; ++q) {
            const unsigned kq = (unsigned)__shfl((int)k, q, kWave);
            if (kq == k) {
                before += q < lane ? 1 : 0;
                after += q > lane ? 1 : 0;
            }
        }
        int base = 0;
        if (v < A.V) base = next[k];
        wave_lds_sync();
        if (v < A.V) {
            A.perm[base + before] = (int)v;
            if (after == 0) next[k] = base + before + 1;
        }
        wave_lds_sync();
    }
}

// Observed curves (and caller weights) in the grouped order; each voxel's group.
__global__ __launch_bounds__(256) void vpet_lb_gather_kernel(LbArgs A) {
    // a thread per (position, frame): coalesced writes, row-contiguous reads
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long p = t / A.F;
    if (p >= A.V) return;
    const int f = (int)(t - p * A.F);
    const long long v = A.perm[p];
    A.ys[t] = A.tacs[(size_t)v * A.F + f];
    if (A.weights) A.ws[t] = A.weights[(size_t)v * A.F + f];
    if (f == 0 && A.out_group) A.out_group[v] = (int)(p / A.S);
}

// One block per group: the Gaussian of each parameter moment-matched to the
// members' mixtures, mean mu_j = avg m_j, variance avg s_j - mu_j^2 (times
// scale^2), in FP64 with a fixed summation order, stored in fp32.
__global__ __launch_bounds__(256) void vpet_lb_fit_kernel(LbArgs A, LbGroup* groups, double scale) {
    __shared__ double red[kRedStride * 4];
    const long long g = blockIdx.x;
    const long long p0 = g * A.S, p1 = min(A.V, p0 + A.S);
    const int D = A.D;
    double s[2 * kLbMaxDims + 1];
#pragma unroll
    for (int q = 0; q < 2 * kLbMaxDims + 1; ++q) s[q] = 0.0;
    for (long long p = p0 + threadIdx.x; p < p1; p += blockDim.x) {
        const long long v = A.perm[p];
        if (A.key[v] >= (unsigned)A.ncell) continue;
        const double* zm = A.zmom + (size_t)v * 2 * D;
        for (int q = 0; q < 2 * D; ++q) s[q] += zm[q];
        s[2 * kLbMaxDims] += 1.0;
    }
    block_sum<2 * kLbMaxDims + 1>(s, red, blockDim.x >> 6);
    if (threadIdx.x == 0) {
        LbGroup G;
        const double cnt = s[2 * kLbMaxDims];
        G.cnt = (int)cnt;
        for (int j = 0; j < kLbMaxDims; ++j) {
            G.mu[j] = 0.0f;
            G.sd[j] = 1.0f;
            if (j < D && cnt > 0.0) {
                const double mu = s[2 * j] / cnt;
                const double var = fmax(s[2 * j + 1] / cnt - mu * mu, 1e-12);
                G.mu[j] = (float)mu;
                G.sd[j] = (float)(sqrt(var) * scale);
            }
        }
        groups[g] = G;
    }
}

// One block per group, four wavefronts, a lane per frame: the mean observed
// curve of the group's valid members (in the grouped order, FP64), the
// reference that the BF16 screen subtracts (padding frames 0).  Wavefront q
// sums the q-th quarter of the members in order, eight members' loads in
// flight at a time; the quarters are added in order.
__global__ __launch_bounds__(256) void vpet_lb_ref_kernel(LbArgs A, double* ref, int ld) {
    __shared__ double part[4][kWave];
    __shared__ long long pcnt[4];
    const long long g = blockIdx.x;
    const int f = threadIdx.x & 63, q = threadIdx.x >> 6;
    const long long p0 = g * A.S, p1 = min(A.V, p0 + A.S), len = p1 - p0;
    const long long a = p0 + len * q / 4, b = p0 + len * (q + 1) / 4;
    double s = 0.0;
    long long cnt = 0;
    if (f < A.F) {
        for (long long p = a; p < b; p += 8) {
            bool ok[8];
            float yv[8];
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                ok[i] = p + i < b && A.key[A.perm[p + i]] < (unsigned)A.ncell;
                yv[i] = ok[i] ? A.ys[(size_t)(p + i) * A.F + f] : 0.0f;
            }
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                if (!ok[i]) continue;
                s += (double)yv[i];
                ++cnt;
            }
        }
    }
    part[q][f] = s;
    if (f == 0) pcnt[q] = cnt;
    __syncthreads();
    if (q == 0 && f < ld) {
        const double t = ((part[0][f] + part[1][f]) + part[2][f]) + part[3][f];
        const long long c = f < A.F ? pcnt[0] + pcnt[1] + pcnt[2] + pcnt[3] : 0;
        ref[(size_t)g * ld + f] = c > 0 ? t / (double)c : 0.0;
    }
}

struct LbBank {
    const LbGroup* groups;
    long long g0;        // first group of this launch
    long long first;     // added to the group index in the Philox counter
    int D, dim_of[kMaxParams];  // head parameter of each model parameter, -1: drawn from the prior
    double share, log_share, log_rest;
    unsigned n_draws, rows_per_group, key0, key1;
    float* theta;        // [groups][rows_per_group][8] (this launch's groups)
    double* x;           // [groups][rows_per_group][ld]
    double* logw;        // [groups][rows_per_group]
    int ld;
    // BF16 screen operands of the rows (bank_bops' layout) and the launch's
    // group reference curves [groups][ld]; null without the contraction screen
    uint16_t* bhi;
    uint16_t* blo;
    const double* ref;
};

// A lane's curve staged in LDS (NaN for an invalid row).
struct StagedRowSink {
    double* s;
    bool valid;
    __device__ __forceinline__ void operator()(int f, int n, const double (&X)[1]) {
        s[f] = valid ? X[0] / (double)n : __builtin_nan("");
    }
};

// Bank row i of model m (list position) of group g = g0 + blockIdx.y: Philox
// stream 3, counters (i, first + g, 3, m << 16 | 0) and (i, first + g, 3,
// m << 16 | 1).
// u0 = ((w0 & 255) | (w1 & 255) << 8 | (w2 & 255) << 16) 2^-24 below the
// share (or an empty group) draws every parameter uniformly from the box;
// otherwise parameter p with a head parameter d gets z_p = mu_d + sd_d n_p,
// theta_p = fp32(exp(z_p)) (invalid outside the box), and a parameter
// without one (k4 under a four-parameter head) is uniform from u_6.  u_p =
// (w_p >> 8) 2^-24 for p < 4, u_4, u_5, u_6 = (v0, v1, v2 >> 8) 2^-24 (the
// second block is drawn for five-parameter models only); normals n_{2q},
// n_{2q+1} = r cos, r sin (2 pi u_{2q+1}), r = sqrt(-2 ln(u_{2q} + 2^-24));
// a uniform draw is theta_p = fp32(lo_p + u wid_p) with lo_p and wid_p = hi_p
// - lo_p in fp32.  log w = -log(a + (1 - a) e^L), L = sum
// over the head's parameters of log N(z_p; mu, sd) - z_p + log(hi_p - lo_p)
// (z_p = log theta_p for a uniform draw); an invalid row has log w = -inf and
// NaN curves.
// A wavefront draws 64 consecutive rows, a lane each, and stages its
// parameter row and then its curve in LDS, so that all of its global writes
// are runs of consecutive elements (a lane writing its own row would send one
// memory request per lane per frame).  With the contraction screen the kernel
// also writes the rows' BF16 operands from the staged curves, as
// bank_bops_kernel would from the stored ones.
template <int KIND>
__global__ __launch_bounds__(kWave) void vpet_lb_bank_kernel(LbBank B, ModelDev md, int m, Tab T, double C0, double h,
                                                             int F, int k0) {
    extern __shared__ double stage[];  // [kWave][ld + 1]: the wavefront's rows, then the reference curve
    const int lane = threadIdx.x;
    const unsigned i = blockIdx.x * kWave + lane;
    const bool live = i < B.n_draws;
    const unsigned ii = live ? i : B.n_draws - 1;
    const long long g = B.g0 + blockIdx.y;
    const LbGroup G = B.groups[g];
    uint32_t w[4], v[4] = {0u, 0u, 0u, 0u};
    const uint32_t gc = (uint32_t)(B.first + g);
    philox10(ii, gc, 3u, (uint32_t)m << 16, B.key0, B.key1, w);
    if (md.np > 4) philox10(ii, gc, 3u, ((uint32_t)m << 16) | 1u, B.key0, B.key1, v);
    const double u0 = (double)((w[0] & 255u) | (w[1] & 255u) << 8 | (w[2] & 255u) << 16) * 0x1p-24;
    double u[7];
#pragma unroll
    for (int q = 0; q < 4; ++q) u[q] = (double)(w[q] >> 8) * 0x1p-24;
#pragma unroll
    for (int q = 0; q < 3; ++q) u[4 + q] = (double)(v[q] >> 8) * 0x1p-24;
    const bool prior = G.cnt == 0 || u0 < B.share;
    float th[kMaxParams];
    double z[kMaxParams];
    bool ok = true;
    double L = 0.0;
#pragma unroll
    for (int p = 0; p < kMaxParams; ++p) {
        th[p] = 0.0f;
        z[p] = 0.0;
    }
    // the Box-Muller normals, once per pair (u_{2q}, u_{2q+1})
    double nrm[2 * 3];
#pragma unroll
    for (int q = 0; q < 3; ++q) {
        nrm[2 * q] = nrm[2 * q + 1] = 0.0;
        if (2 * q < md.np) {
            const double r = sqrt(-2.0 * log_pos(u[2 * q] + 0x1p-24));
            double sn, cs;
            sincospi(2.0 * u[2 * q + 1], &sn, &cs);
            nrm[2 * q] = r * cs;
            nrm[2 * q + 1] = r * sn;
        }
    }
    // log wid_p (lanes 0-7) and log sd_d (lanes 8-15), one logarithm per
    // lane, read back per parameter
    double lgv;
    {
        float a = 1.0f;
#pragma unroll
        for (int p = 0; p < kMaxParams; ++p)
            if (lane == p) a = md.wid[p];
#pragma unroll
        for (int d = 0; d < kLbMaxDims; ++d)
            if (lane == 8 + d) a = G.sd[d];
        lgv = log((double)a);
    }
#pragma unroll
    for (int p = 0; p < kMaxParams; ++p) {
        if (p >= md.np) break;
        const double lo = (double)md.lo[p], wid = (double)md.wid[p];
        const int d = B.dim_of[p];
        if (prior || d < 0 || wid == 0.0) {
            th[p] = (float)(lo + (prior || wid == 0.0 ? u[p] : u[6]) * wid);
            z[p] = log((double)th[p]);
        } else {
            z[p] = (double)G.mu[d] + (double)G.sd[d] * nrm[p];
            th[p] = (float)exp_series(z[p]);
            ok = ok && th[p] >= md.lo[p] && (double)th[p] <= lo + wid;
        }
        if (d >= 0 && wid > 0.0 && G.cnt > 0) {
            const double t = (z[p] - (double)G.mu[d]) / (double)G.sd[d];
            L += -0.5 * t * t - lane_f64(lgv, 8 + d) - 0.9189385332046727 - z[p] + lane_f64(lgv, p);
        }
    }
    double lw = 0.0;
    if (G.cnt > 0) {
        if (!isfinite(L)) {
            lw = L > 0.0 ? -__builtin_inf() : -B.log_share;  // q / p = 0: weight 1 / a
        } else if (B.share == 0.0) {
            lw = -L;
        } else {
            const double x = B.log_share, y = B.log_rest + L;  // -logaddexp(x, y)
            const double mxy = fmax(x, y);
            lw = -(mxy + log1p(exp(-fabs(x - y))));
        }
    }
    if (!ok) lw = -__builtin_inf();
    // the wavefront's rows are consecutive: row0 + r for r < nlive
    const int ld = B.ld;
    const int nlive = (int)min(B.n_draws - blockIdx.x * kWave, (unsigned)kWave);
    const size_t row0 = (size_t)blockIdx.y * B.rows_per_group + (size_t)m * B.n_draws + blockIdx.x * kWave;
    if (live) B.logw[row0 + lane] = lw;
    if (B.bhi && lane < ld) stage[kWave * (ld + 1) + lane] = B.ref[(size_t)blockIdx.y * ld + lane];
    {  // parameter rows through LDS, written out as consecutive floats
        float* tf = reinterpret_cast<float*>(stage);
#pragma unroll
        for (int j = 0; j < VPET_PSTRIDE; ++j) tf[lane * VPET_PSTRIDE + j] = __builtin_nanf("");
        for (int q = 0; q < md.np; ++q) tf[lane * VPET_PSTRIDE + md.slot[q]] = th[q];
        __syncthreads();
        float* to = B.theta + row0 * VPET_PSTRIDE;
#pragma unroll
        for (int k = 0; k < VPET_PSTRIDE; ++k) {
            const int e = k * kWave + lane;
            if (e < nlive * VPET_PSTRIDE) to[e] = tf[e];
        }
        __syncthreads();
    }
    if (!ok) {  // an in-box stand-in keeps the recursion finite; the row's curve is NaN
        for (int p = 0; p < md.np; ++p) th[p] = md.lo[p];
        th[1] = md.lo[1] + md.wid[1];
    }
    double* mine = stage + lane * (ld + 1);
    for (int f = F; f < ld; ++f) mine[f] = 0.0;
    StagedRowSink sink{mine, ok};
    constexpr int NE = ModelTraits<KIND>::NE;
    DrawState<NE, 1> s;
    setup<KIND, NE, 1>(th, h, C0, s, 0);
    simulate_draws<KIND, 1>(T, F, k0, s, sink);
    __syncthreads();
    // the rows leave as consecutive elements: lane + 64 k of the wavefront's
    // kWave x ld block, (r, f) advanced by (64 / ld, 64 % ld) per step; ld is
    // a multiple of 8 and r stays below kWave
    {
        double* xo = B.x + row0 * (size_t)ld;
        const int dr = kWave / ld, df = kWave % ld;
        int r = lane / ld, f = lane % ld;
        for (int k = 0; k < ld; k += 4) {
            double v[4];
            bool w[4];
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                w[j] = r < nlive;
                v[j] = stage[r * (ld + 1) + f];
                r += dr;
                f += df;
                if (f >= ld) {
                    f -= ld;
                    ++r;
                }
            }
#pragma unroll
            for (int j = 0; j < 4; ++j)
                if (w[j]) xo[(size_t)(k + j) * kWave + lane] = v[j];
        }
    }
    if (B.bhi) {  // the screen operands of bank_bops, pairs of frames per lane
        const int hp = ld >> 1, dr = kWave / hp, df = kWave % hp;
        const double* rs = stage + kWave * (ld + 1);  // the group's reference curve
        uint32_t* bh = reinterpret_cast<uint32_t*>(B.bhi) + row0 * (size_t)ld;
        uint32_t* bl = reinterpret_cast<uint32_t*>(B.blo) + row0 * (size_t)ld;
        int r = lane / hp, pr = lane % hp;
        for (int k = 0; k < hp; k += 4) {
            double x0[4], x1[4];
            int o[4];
            bool w[4];
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                w[j] = r < nlive;
                o[j] = r * ld + pr;
                x0[j] = stage[r * (ld + 1) + 2 * pr] - rs[2 * pr];
                x1[j] = stage[r * (ld + 1) + 2 * pr + 1] - rs[2 * pr + 1];
                r += dr;
                pr += df;
                if (pr >= hp) {
                    pr -= hp;
                    ++r;
                }
            }
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                if (!w[j]) continue;
                split_bf16x2(x0[j], x1[j], bh[o[j]], bl[o[j]]);
                split_bf16x2(x0[j] * x0[j], x1[j] * x1[j], bh[o[j] + hp], bl[o[j] + hp]);
            }
        }
    }
}

// Table staging for the allocation-free entry point: 1 KB of table bytes per
// launch, carried in the kernel argument (copied by the runtime at launch, so
// no host staging buffer has to outlive the call).
constexpr int kStageWords = 128;
struct StageChunk {
    unsigned long long w[kStageWords];
};
__global__ __launch_bounds__(kStageWords) void vpet_stage_kernel(StageChunk c, unsigned long long* dst, int nwords) {
    if ((int)threadIdx.x < nwords) dst[threadIdx.x] = c.w[threadIdx.x];
}

}  // namespace

// Device memory of vpet_abc_infer_noalloc: the draw-independent tables of the
// call (input nodes, frame sums, frame lengths; at most 256 KB), one copy per
// GPU for the life of the process.  Host code must not use this name as an
// address: it reaches the array only through the pointer hipGetSymbolAddress
// returns for the current device.
static __device__ __align__(256) unsigned char scratch[256 * 1024];

namespace {

// ===========================================================================
// Host side.
// ===========================================================================
thread_local std::string g_err;

int fail(int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

int hip_fail(hipError_t e, const char* what) {
    return fail(VPET_E_HIP, "%s: %s", what, hipGetErrorString(e));
}

// Draw-independent tables, FP64 on the host.
struct HostTab {
    int K = 0, F = 0, k0 = 0, kend = 0;
    double h = 0.0, C0 = 0.0;
    std::vector<double> C, fr;
    std::vector<int> nf;
};

int make_tables(const float* input_fn, const float* frame_times, vpet_grid g, double lambda, HostTab& T) {
    if (!input_fn || !frame_times) return fail(VPET_E_ARG, "input_fn and frame_times must not be NULL");
    if (!(std::isfinite(g.dt) && g.dt > 0.0f)) return fail(VPET_E_GRID, "grid.dt must be finite and > 0");
    if (g.n_nodes < 2 || g.n_nodes > VPET_MAX_NODES)
        return fail(g.n_nodes > VPET_MAX_NODES ? VPET_E_LIMIT : VPET_E_GRID, "grid.n_nodes %d outside [2, %d]",
                    g.n_nodes, VPET_MAX_NODES);
    if (g.n_frames < 1 || g.n_frames > VPET_MAX_FRAMES)
        return fail(g.n_frames > VPET_MAX_FRAMES ? VPET_E_LIMIT : VPET_E_GRID, "grid.n_frames %d outside [1, %d]",
                    g.n_frames, VPET_MAX_FRAMES);
    T.K = g.n_nodes - 1;
    T.F = g.n_frames;
    T.h = (double)g.dt;
    for (int k = 0; k <= T.K; ++k)
        if (!std::isfinite(input_fn[k])) return fail(VPET_E_ARG, "input_fn[%d] is not finite", k);
    std::vector<int> kf(T.F + 1);
    for (int f = 0; f <= T.F; ++f) {
        const double tau = (double)frame_times[f];
        if (!std::isfinite(tau)) return fail(VPET_E_GRID, "frame_times[%d] is not finite", f);
        const double kd = std::nearbyint(tau / T.h);
        if (std::fabs(kd * T.h - tau) > 1e-6 * std::fmax(1.0, std::fabs(tau)))
            return fail(VPET_E_GRID, "frame bound %g is not on the %g-min grid", tau, T.h);
        if (kd < 0.0 || kd > (double)T.K)
            return fail(VPET_E_GRID, "frame bound %g lies outside the grid [0, %g]", tau, T.K * T.h);
        kf[f] = (int)kd;
        if (f > 0 && kf[f] <= kf[f - 1]) return fail(VPET_E_GRID, "frame bounds must increase strictly");
    }
    T.k0 = kf[0];
    T.kend = kf[T.F];
    T.C0 = (double)input_fn[0];
    std::vector<double> Cn(T.kend + 1), Q(T.kend + 1);
    for (int k = 0; k <= T.kend; ++k) Cn[k] = (double)input_fn[k];
    Q[0] = 0.0;
    for (int k = 0; k < T.kend; ++k) Q[k + 1] = Q[k] + 0.5 * T.h * (Cn[k] + Cn[k + 1]);
    T.C.assign(Cn.begin(), Cn.begin() + T.kend + 1);
    T.fr.assign(4 * (size_t)T.F, 0.0);
    T.nf.assign(T.F, 0);
    for (int f = 0; f < T.F; ++f) {
        const int a = kf[f], b = kf[f + 1];
        double ss = 0.5 * (Q[a] + Q[b]), pp = 0.5 * (Cn[a] + Cn[b]), rr = 0.0;
        for (int k = a + 1; k < b; ++k) {
            ss += Q[k];
            pp += Cn[k];
        }
        for (int k = a; k < b; ++k) rr += Cn[k];
        const double dt = (double)(b - a) * T.h;
        const double tmid = 0.5 * (double)(a + b) * T.h;
        T.fr[4 * f + 0] = ss;
        T.fr[4 * f + 1] = pp;
        T.fr[4 * f + 2] = rr;
        T.fr[4 * f + 3] = dt * std::exp(-lambda * tmid);
        T.nf[f] = b - a;
    }
    return VPET_OK;
}

// Model kinds in bit order; -1 for unknown bits or a mix of the plasma-input
// family (1TCM, 2TCMs) and the reference-tissue family (MRTM, lp-ntPET),
// whose inputs differ.
int model_list(uint32_t model_id, int kinds[kMaxModels]) {
    constexpr uint32_t plasma = VPET_M_1TCM | VPET_M_2TCM_IRR | VPET_M_2TCM_REV;
    constexpr uint32_t reference = VPET_M_MRTM | VPET_M_LPNTPET;
    if (model_id == 0u || (model_id & ~(plasma | reference)) != 0u) return -1;
    if ((model_id & plasma) && (model_id & reference)) return -1;
    int M = 0;
    for (uint32_t b = 1u; b <= VPET_M_LPNTPET; b <<= 1)
        if (model_id & b) kinds[M++] = (int)b;
    return M;
}

bool is_reference(int kind) { return kind == KIND_MRTM || kind == KIND_LPNT; }

int fill_reference_model(int kind, const double* box, ModelDev& md) {
    md = ModelDev{};
    md.kind = kind;
    md.np = kind == KIND_MRTM ? 3 : 7;
    md.rel_tp = kind == KIND_LPNT;
    for (int j = 0; j < md.np; ++j) {
        const double lo = box[2 * j], hi = box[2 * j + 1];
        if (!(std::isfinite(lo) && std::isfinite(hi))) return fail(VPET_E_ARG, "prior box slot %d is not finite", j);
        if (lo > hi) return fail(VPET_E_ARG, "prior box slot %d has lo > hi", j);
        if (lo < 0.0) return fail(VPET_E_ARG, "prior box slot %d must be >= 0", j);
        md.slot[j] = j;
        md.lo[j] = (float)lo;
        md.wid[j] = (float)(hi - lo);
    }
    if (!(box[2 * VPET_SLOT_K2A] > 0.0)) return fail(VPET_E_ARG, "k2a prior needs lo > 0");
    if (kind == KIND_LPNT) {
        // tP in [tD + lo, hi]: lo is an offset; the interval must be non-empty
        // for every tD in its box
        const double off = box[2 * VPET_SLOT_TP], hi = box[2 * VPET_SLOT_TP + 1];
        if (!(off > 0.0)) return fail(VPET_E_ARG, "the tP offset after tD (box lo) must be > 0");
        if (!(box[2 * VPET_SLOT_TD + 1] + off <= hi))
            return fail(VPET_E_ARG, "tP box: tD_hi + offset must not exceed tP_hi");
        if (!(box[2 * VPET_SLOT_ALPHA] > 0.0)) return fail(VPET_E_ARG, "alpha prior needs lo > 0");
        md.lo[VPET_SLOT_TP] = (float)off;
        md.wid[VPET_SLOT_TP] = (float)hi;
    }
    return VPET_OK;
}

int fill_model(int kind, const double* box, ModelDev& md) {
    if (is_reference(kind)) return fill_reference_model(kind, box, md);
    static const int s1[3] = {VPET_SLOT_K1, VPET_SLOT_K2, VPET_SLOT_VB};
    static const int s2[4] = {VPET_SLOT_K1, VPET_SLOT_K2, VPET_SLOT_K3, VPET_SLOT_VB};
    static const int s3[5] = {VPET_SLOT_K1, VPET_SLOT_K2, VPET_SLOT_K3, VPET_SLOT_K4, VPET_SLOT_VB};
    const int* sl = kind == KIND_1TCM ? s1 : (kind == KIND_IRR ? s2 : s3);
    md = ModelDev{};
    md.kind = kind;
    md.np = kind == KIND_1TCM ? 3 : (kind == KIND_IRR ? 4 : 5);
    for (int j = 0; j < md.np; ++j) {
        const int s = sl[j];
        const double lo = box[2 * s], hi = box[2 * s + 1];
        if (!(std::isfinite(lo) && std::isfinite(hi))) return fail(VPET_E_ARG, "prior box slot %d is not finite", s);
        if (lo > hi) return fail(VPET_E_ARG, "prior box slot %d has lo > hi", s);
        if (lo < 0.0) return fail(VPET_E_ARG, "prior box slot %d must be >= 0", s);
        if (s == VPET_SLOT_VB && !(hi < 1.0)) return fail(VPET_E_ARG, "vB must stay below 1");
        md.slot[j] = s;
        md.lo[j] = (float)lo;
        md.wid[j] = (float)(hi - lo);
    }
    if (kind != KIND_1TCM && !(box[2 * VPET_SLOT_K2] + box[2 * VPET_SLOT_K3] > 0.0))
        return fail(VPET_E_ARG, "2TCM prior needs k2_lo + k3_lo > 0");
    if (kind == KIND_REV && !(box[2 * VPET_SLOT_K3] > 0.0))
        return fail(VPET_E_ARG, "reversible 2TCM prior needs k3_lo > 0");
    return VPET_OK;
}

// Per-device ring of (pinned host, device) table slots.
constexpr int kSlots = 8;
constexpr size_t kSlotBytes = 256 * 1024;

struct DevCtx {
    std::mutex mu;
    bool ready = false;
    char* dbuf = nullptr;
    char* hbuf = nullptr;
    hipEvent_t ev[kSlots];
    int next = 0;
};
DevCtx g_ctx[64];

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// Uploads T into a slot and returns device pointers; the caller holds ctx.mu
// until it has recorded ctx.ev[slot] after its launch.
// Byte layout of the tables in device memory: C (FP64), the per-frame sums
// (FP64) and the frame lengths in nodes (int32), each 256-byte aligned.
struct TabLayout {
    size_t offC, offF, offN, bytes;
};
TabLayout tab_layout(const HostTab& T) {
    TabLayout L;
    L.offC = 0;
    L.offF = align256(L.offC + sizeof(double) * T.C.size());
    L.offN = align256(L.offF + sizeof(double) * T.fr.size());
    L.bytes = align256(L.offN + sizeof(int) * T.nf.size());
    return L;
}

int upload_tables(DevCtx& ctx, const HostTab& T, hipStream_t st, Tab& tab, int& slot) {
    if (!ctx.ready) {
        hipError_t e = hipMalloc((void**)&ctx.dbuf, kSlots * kSlotBytes);
        if (e != hipSuccess) return fail(VPET_E_NOMEM, "table buffer: %s", hipGetErrorString(e));
        e = hipHostMalloc((void**)&ctx.hbuf, kSlots * kSlotBytes, hipHostMallocDefault);
        if (e != hipSuccess) return fail(VPET_E_NOMEM, "pinned table buffer: %s", hipGetErrorString(e));
        for (int s = 0; s < kSlots; ++s) {
            e = hipEventCreateWithFlags(&ctx.ev[s], hipEventDisableTiming);
            if (e != hipSuccess) return hip_fail(e, "hipEventCreate");
        }
        ctx.ready = true;
    }
    const TabLayout L = tab_layout(T);
    const size_t offC = L.offC, offF = L.offF, offN = L.offN, bytes = L.bytes;
    if (bytes > kSlotBytes) return fail(VPET_E_LIMIT, "tables need %zu bytes (> %zu)", bytes, kSlotBytes);
    slot = ctx.next;
    ctx.next = (ctx.next + 1) % kSlots;
    hipError_t e = hipEventSynchronize(ctx.ev[slot]);
    if (e != hipSuccess) return hip_fail(e, "hipEventSynchronize");
    char* hs = ctx.hbuf + slot * kSlotBytes;
    char* ds = ctx.dbuf + slot * kSlotBytes;
    if (!T.C.empty()) std::memcpy(hs + offC, T.C.data(), sizeof(double) * T.C.size());
    std::memcpy(hs + offF, T.fr.data(), sizeof(double) * T.fr.size());
    std::memcpy(hs + offN, T.nf.data(), sizeof(int) * T.nf.size());
    e = hipMemcpyAsync(ds, hs, bytes, hipMemcpyHostToDevice, st);
    if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync(tables)");
    tab.C = reinterpret_cast<const double*>(ds + offC);
    tab.fr = reinterpret_cast<const double*>(ds + offF);
    tab.nf = reinterpret_cast<const int*>(ds + offN);
    return VPET_OK;
}

// Uploads `bytes` of host data into a slot (same ring and locking rules as
// upload_tables).
int upload_blob(DevCtx& ctx, const void* data, size_t bytes, hipStream_t st, const void** dptr, int& slot) {
    if (!ctx.ready) {
        Tab t;
        HostTab T;
        T.fr.assign(4, 0.0);
        T.nf.assign(1, 0);
        int rc = upload_tables(ctx, T, st, t, slot);  // allocates the ring
        if (rc != VPET_OK) return rc;
        hipError_t e = hipEventRecord(ctx.ev[slot], st);
        if (e != hipSuccess) return hip_fail(e, "hipEventRecord");
    }
    if (bytes > kSlotBytes) return fail(VPET_E_LIMIT, "table of %zu bytes exceeds %zu", bytes, kSlotBytes);
    slot = ctx.next;
    ctx.next = (ctx.next + 1) % kSlots;
    hipError_t e = hipEventSynchronize(ctx.ev[slot]);
    if (e != hipSuccess) return hip_fail(e, "hipEventSynchronize");
    char* hs = ctx.hbuf + slot * kSlotBytes;
    char* ds = ctx.dbuf + slot * kSlotBytes;
    std::memcpy(hs, data, bytes);
    e = hipMemcpyAsync(ds, hs, bytes, hipMemcpyHostToDevice, st);
    if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync(table)");
    *dptr = ds;
    return VPET_OK;
}

// Stream-ordered scratch comes from the device's default memory pool; once
// per device the pool is told to keep up to 32 GiB of freed memory for reuse
// (with the default threshold of 0 it returns freed memory to the system at
// every synchronisation, and a call with banks of several GiB paid for mapping
// them again each time).
std::atomic<bool> g_pool_kept[64];

void keep_pool(int dev) {
    if (g_pool_kept[dev].exchange(true)) return;
    hipMemPool_t pool;
    if (hipDeviceGetDefaultMemPool(&pool, dev) == hipSuccess) {
        uint64_t thr = 32ull << 30;
        (void)hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &thr);
    }
}

int current_device(int* dev) {
    hipError_t e = hipGetDevice(dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    if (*dev < 0 || *dev >= 64) return fail(VPET_E_HIP, "device ordinal %d out of range", *dev);
    keep_pool(*dev);
    return VPET_OK;
}

int current_ctx(DevCtx** out) {
    int dev = 0;
    const int rc = current_device(&dev);
    if (rc != VPET_OK) return rc;
    *out = &g_ctx[dev];
    return VPET_OK;
}

// Allocation-free table staging (vpet_abc_infer_noalloc).  The address of
// `scratch` on a device is looked up once, with that device current, and kept;
// every call on the device then writes its tables there in stream order.
std::mutex g_noalloc_mu;
void* g_noalloc_ptr[64];

int noalloc_scratch(unsigned char** out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    if (dev < 0 || dev >= 64) return fail(VPET_E_HIP, "device ordinal %d out of range", dev);
    std::lock_guard<std::mutex> lock(g_noalloc_mu);
    if (!g_noalloc_ptr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
        if (!p) return fail(VPET_E_HIP, "hipGetSymbolAddress(scratch) returned NULL");
        g_noalloc_ptr[dev] = p;
    }
    *out = static_cast<unsigned char*>(g_noalloc_ptr[dev]);
    return VPET_OK;
}

// n bytes of host data to dst in 1 KB kernel arguments; the last word of a
// chunk is zero-padded (dst must have room up to the next 8-byte boundary).
int stage_bytes(const void* src, size_t n, unsigned char* dst, hipStream_t st) {
    const unsigned char* s = static_cast<const unsigned char*>(src);
    for (size_t off = 0; off < n; off += sizeof(StageChunk)) {
        StageChunk c;
        const size_t len = std::min(n - off, sizeof(StageChunk));
        std::memset(&c, 0, sizeof c);
        std::memcpy(&c, s + off, len);
        hipLaunchKernelGGL(vpet_stage_kernel, dim3(1), dim3(kStageWords), 0, st, c,
                           reinterpret_cast<unsigned long long*>(dst + off), (int)((len + 7) / 8));
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return hip_fail(e, "table staging launch");
    }
    return VPET_OK;
}

int stage_tables_noalloc(const HostTab& T, hipStream_t st, Tab& tab) {
    const TabLayout L = tab_layout(T);
    if (L.bytes > sizeof(scratch))
        return fail(VPET_E_LIMIT, "tables need %zu bytes (> %zu, the allocation-free buffer)", L.bytes,
                    sizeof(scratch));
    unsigned char* base = nullptr;
    int rc = noalloc_scratch(&base);
    if (rc != VPET_OK) return rc;
    if (!T.C.empty() && (rc = stage_bytes(T.C.data(), sizeof(double) * T.C.size(), base + L.offC, st)) != VPET_OK)
        return rc;
    if ((rc = stage_bytes(T.fr.data(), sizeof(double) * T.fr.size(), base + L.offF, st)) != VPET_OK) return rc;
    if ((rc = stage_bytes(T.nf.data(), sizeof(int) * T.nf.size(), base + L.offN, st)) != VPET_OK) return rc;
    tab.C = reinterpret_cast<const double*>(base + L.offC);
    tab.fr = reinterpret_cast<const double*>(base + L.offF);
    tab.nf = reinterpret_cast<const int*>(base + L.offN);
    return VPET_OK;
}

// Frame bounds of the bank form (validated) and the weights' decay factors
// omega_f = dt_f exp(-lambda tmid_f) (the input function is not needed).
int bank_omega(const float* frame_times, vpet_grid grid, double decay_lambda, std::vector<double>& omega) {
    if (!frame_times) return fail(VPET_E_ARG, "frame_times must not be NULL");
    if (!(std::isfinite(grid.dt) && grid.dt > 0.0f)) return fail(VPET_E_GRID, "grid.dt must be finite and > 0");
    if (grid.n_nodes < 2 || grid.n_frames < 1) return fail(VPET_E_GRID, "grid needs n_nodes >= 2, n_frames >= 1");
    if (grid.n_frames > VPET_BANK_MAX_FRAMES)
        return fail(VPET_E_LIMIT, "the bank form supports up to %d frames", VPET_BANK_MAX_FRAMES);
    const double h = (double)grid.dt, lambda = decay_lambda > 0.0 ? decay_lambda : std::log(2.0) / 109.8;
    const int F = grid.n_frames, K = grid.n_nodes - 1;
    omega.assign(F, 0.0);
    int kprev = -1;
    for (int f = 0; f <= F; ++f) {
        const double tau = (double)frame_times[f];
        if (!std::isfinite(tau)) return fail(VPET_E_GRID, "frame_times[%d] is not finite", f);
        const double kd = std::nearbyint(tau / h);
        if (std::fabs(kd * h - tau) > 1e-6 * std::fmax(1.0, std::fabs(tau)))
            return fail(VPET_E_GRID, "frame bound %g is not on the %g-min grid", tau, h);
        if (kd < 0.0 || kd > (double)K) return fail(VPET_E_GRID, "frame bound %g lies outside the grid", tau);
        const int k = (int)kd;
        if (f > 0) {
            if (k <= kprev) return fail(VPET_E_GRID, "frame bounds must increase strictly");
            omega[f - 1] = (double)(k - kprev) * h * std::exp(-lambda * 0.5 * (double)(k + kprev) * h);
        }
        kprev = k;
    }
    return VPET_OK;
}

int pow2_at_least(int x) {
    int p = 1;
    while (p < x) p <<= 1;
    return p;
}

// Keys the re-ranking select holds in LDS (a power of two, at most the list
// capacity).  About 4 n keys at or below tau are expected; a fuller buffer is
// first pruned to the smallest keys (about 1.25 n) and overflows into the
// exact fallback only if that fails.  8 n while that is at most 1024 keys
// (LDS then does not limit the kernel's occupancy); beyond, the least that
// still holds the outputs' staging past the n accepted keys (6 n keys in all
// with importance weights, 5 n + 1 without).
int select_key_buffer(int cap, int n, bool weighted) {
    const int want = pow2_at_least(8 * n) <= 1024 ? 8 * n : (weighted ? 6 * n : 5 * n + 1);
    return std::min(cap, std::max(512, pow2_at_least(want)));
}

}  // namespace

// ===========================================================================
// C ABI.
// ===========================================================================
namespace {
// BF16 hi/lo operands B_g = [x_g, x_g^2] of the first `rows` bank rows.
void bank_bops(BankArgs A, unsigned rows, hipStream_t st, int ld) {
    A.n_tot = rows;
    const dim3 gb((unsigned)(((unsigned long long)rows * (unsigned)(ld / 2) + 255) / 256)), b256(256);
    switch (ld) {
        case 8: hipLaunchKernelGGL((vpet_bank_bops_kernel<8>), gb, b256, 0, st, A); break;
        case 16: hipLaunchKernelGGL((vpet_bank_bops_kernel<16>), gb, b256, 0, st, A); break;
        case 24: hipLaunchKernelGGL((vpet_bank_bops_kernel<24>), gb, b256, 0, st, A); break;
        case 32: hipLaunchKernelGGL((vpet_bank_bops_kernel<32>), gb, b256, 0, st, A); break;
        case 40: hipLaunchKernelGGL((vpet_bank_bops_kernel<40>), gb, b256, 0, st, A); break;
        default: hipLaunchKernelGGL((vpet_bank_bops_kernel<48>), gb, b256, 0, st, A); break;
    }
}

// One voxel chunk of the bank form: reset, (BF16 voxel operands,) pilot,
// scan, select and the exact fallback; mark(0) / mark(1) bracket the scan.
template <class Mark>
void bank_chunk(const BankArgs& Q, hipStream_t st, int ld, bool l1, bool mfma, size_t lds, size_t fb_lds,
                int fb_waves, Mark& mark) {
    const dim3 lanes((unsigned)((Q.V + 255) / 256)), b256(256), per_voxel((unsigned)Q.V), b64(64);
    const dim3 mblocks((unsigned)((Q.V + kMfmaVox - 1) / kMfmaVox));
    const dim3 fb_grid((unsigned)std::min<long long>(Q.V, 2048)), fb_block(64 * fb_waves), one(1);
#define VPET_BANK_LAUNCH(LDV, L1V)                                                                        \
    do {                                                                                                  \
        hipLaunchKernelGGL(vpet_bank_reset_kernel, one, one, 0, st, Q);                                   \
        if (mfma) {                                                                                       \
            hipLaunchKernelGGL((vpet_bank_aops_kernel<LDV>), lanes, b256, 0, st, Q);                      \
            launch_mfma<2 * LDV, true>(mblocks, st, Q);                                                   \
            mark(0);                                                                                      \
            launch_mfma<2 * LDV, false>(mblocks, st, Q);                                                  \
            mark(1);                                                                                      \
            if (Q.bank_logw)                                                                              \
                hipLaunchKernelGGL((vpet_bank_select_kernel<LDV, L1V, true, true>), per_voxel, b64, lds, st, Q); \
            else                                                                                          \
                hipLaunchKernelGGL((vpet_bank_select_kernel<LDV, L1V, true, false>), per_voxel, b64, lds, st, Q); \
        } else {                                                                                          \
            hipLaunchKernelGGL((vpet_bank_scan_kernel<LDV, L1V, true>), lanes, b256, 0, st, Q);           \
            mark(0);                                                                                      \
            hipLaunchKernelGGL((vpet_bank_scan_kernel<LDV, L1V, false>), lanes, b256, 0, st, Q);          \
            mark(1);                                                                                      \
            if (Q.bank_logw)                                                                              \
                hipLaunchKernelGGL((vpet_bank_select_kernel<LDV, L1V, false, true>), per_voxel, b64, lds, st, Q); \
            else                                                                                          \
                hipLaunchKernelGGL((vpet_bank_select_kernel<LDV, L1V, false, false>), per_voxel, b64, lds, st, Q); \
        }                                                                                                 \
        hipLaunchKernelGGL((vpet_bank_fallback_kernel<LDV, L1V>), fb_grid, fb_block, fb_lds, st, Q);      \
    } while (0)
    const int sel = (ld / 8) * 2 + (l1 ? 1 : 0);
    switch (sel) {
        case 2: VPET_BANK_LAUNCH(8, false); break;
        case 3: VPET_BANK_LAUNCH(8, true); break;
        case 4: VPET_BANK_LAUNCH(16, false); break;
        case 5: VPET_BANK_LAUNCH(16, true); break;
        case 6: VPET_BANK_LAUNCH(24, false); break;
        case 7: VPET_BANK_LAUNCH(24, true); break;
        case 8: VPET_BANK_LAUNCH(32, false); break;
        case 9: VPET_BANK_LAUNCH(32, true); break;
        case 10: VPET_BANK_LAUNCH(40, false); break;
        case 11: VPET_BANK_LAUNCH(40, true); break;
        case 12: VPET_BANK_LAUNCH(48, false); break;
        default: VPET_BANK_LAUNCH(48, true); break;
    }
#undef VPET_BANK_LAUNCH
}

}  // namespace

extern "C" {

const char* vpet_abc_last_error(void) { return g_err.c_str(); }

int vpet_abc_version(void) { return VPET_VERSION_NUMBER; }

int vpet_abc_accept_count(int64_t n_total, double accept_frac, int64_t* out_n) {
    if (!out_n) return fail(VPET_E_ARG, "out_n must not be NULL");
    if (n_total < 1) return fail(VPET_E_ARG, "n_total must be >= 1");
    if (!(accept_frac > 0.0 && accept_frac <= 1.0)) return fail(VPET_E_ARG, "accept_frac must lie in (0, 1]");
    const double v = std::floor((double)n_total * accept_frac + 1e-6);
    if (v < 1.0) return fail(VPET_E_ARG, "n = floor(N p) = 0: accept at least one draw");
    *out_n = v > (double)n_total ? n_total : (int64_t)v;
    return VPET_OK;
}

int vpet_abc_simulate(uint32_t model_id, const float* theta, int64_t n, const float* input_fn,
                      const float* frame_times, vpet_grid grid, float* out_tacs, void* hip_stream) {
    int kinds[kMaxModels];
    const int M = model_list(model_id, kinds);
    if (M != 1) return fail(VPET_E_MODEL, "simulate needs exactly one known model bit (got 0x%x)", model_id);
    if (n < 0) return fail(VPET_E_ARG, "n must be >= 0");
    HostTab T;
    int rc = make_tables(input_fn, frame_times, grid, 0.0, T);
    if (rc != VPET_OK) return rc;
    if (n == 0) return VPET_OK;
    if (!theta || !out_tacs) return fail(VPET_E_ARG, "theta and out_tacs must not be NULL");
    DevCtx* ctx;
    if ((rc = current_ctx(&ctx)) != VPET_OK) return rc;
    hipStream_t st = (hipStream_t)hip_stream;
    std::lock_guard<std::mutex> lock(ctx->mu);
    Tab tab;
    int slot;
    if ((rc = upload_tables(*ctx, T, st, tab, slot)) != VPET_OK) return rc;
    const int threads = 256;
    for (long long base = 0; base < n; base += (1LL << 30)) {
        const long long cnt = std::min<long long>(n - base, 1LL << 30);
        const unsigned blocks = (unsigned)((cnt + threads - 1) / threads);
        const float* th = theta + (size_t)base * VPET_PSTRIDE;
        float* out = out_tacs + (size_t)base * T.F;
#define VPET_SIM(KD)                                                                                  \
    hipLaunchKernelGGL(vpet_simulate_kernel<KD>, dim3(blocks), dim3(threads), 0, st, th, cnt, tab, T.C0, T.h, \
                       T.F, T.k0, out)
        switch (kinds[0]) {
            case KIND_1TCM: VPET_SIM(KIND_1TCM); break;
            case KIND_IRR: VPET_SIM(KIND_IRR); break;
            case KIND_REV: VPET_SIM(KIND_REV); break;
            case KIND_MRTM: VPET_SIM(KIND_MRTM); break;
            default: VPET_SIM(KIND_LPNT); break;
        }
#undef VPET_SIM
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return hip_fail(e, "simulate launch");
    }
    hipError_t e = hipEventRecord(ctx->ev[slot], st);
    if (e != hipSuccess) return hip_fail(e, "hipEventRecord");
    return VPET_OK;
}

// vpet_abc_infer and its allocation-free variant: identical kernels; the
// tables go to the pooled slots or to `scratch`.
static int infer_entry(bool noalloc, const float* tacs, int64_t n_voxels, const float* frame_times,
                       const float* input_fn, vpet_grid grid, uint32_t model_id, const double* prior_box,
                       int64_t n_draws, double accept_frac, uint64_t seed, float* out_moments,
                       float* out_model_prob, const vpet_abc_opts* opts, void* hip_stream) {
    int kinds[kMaxModels];
    const int M = model_list(model_id, kinds);
    if (M < 1) return fail(VPET_E_MODEL, "unknown or empty model bitmask 0x%x", model_id);
    if (is_reference(kinds[0]))
        return fail(VPET_E_MODEL, "reference-tissue models run in the shared-bank form (vpet_abc_infer_bank)");
    if (n_voxels < 0) return fail(VPET_E_ARG, "n_voxels must be >= 0");
    if (!prior_box) return fail(VPET_E_ARG, "prior_box must not be NULL");
    if (n_draws < 1) return fail(VPET_E_ARG, "n_draws must be >= 1");
    if ((double)M * (double)n_draws > 4294967295.0)
        return fail(VPET_E_LIMIT, "M * n_draws must stay below 2^32");
    vpet_abc_opts o{};
    if (opts) o = *opts;
    if (o.voxel_offset < 0 || (double)o.voxel_offset + (double)n_voxels > 4294967296.0)
        return fail(VPET_E_ARG, "voxel indices must lie in [0, 2^32)");
    if (o.distance != 0 && o.distance != 1) return fail(VPET_E_ARG, "opts.distance must be 0 (L2) or 1 (L1)");
    if (!(std::isfinite(o.decay_lambda) && o.decay_lambda >= 0.0))
        return fail(VPET_E_ARG, "opts.decay_lambda must be finite and >= 0");
    if (!(std::isfinite(o.weight_floor_frac) && o.weight_floor_frac >= 0.0f))
        return fail(VPET_E_ARG, "opts.weight_floor_frac must be finite and >= 0");
    if (o.waves_per_voxel != 0 && o.waves_per_voxel != 1 && o.waves_per_voxel != 2 && o.waves_per_voxel != 4)
        return fail(VPET_E_ARG, "opts.waves_per_voxel must be 0, 1, 2 or 4");
    int64_t n_acc = 0;
    int rc = vpet_abc_accept_count((int64_t)M * n_draws, accept_frac, &n_acc);
    if (rc != VPET_OK) return rc;
    if (n_acc > VPET_MAX_ACCEPT)
        return fail(VPET_E_LIMIT, "n = %lld accepted draws exceeds VPET_MAX_ACCEPT = %d", (long long)n_acc,
                    VPET_MAX_ACCEPT);
    InferArgs P{};
    for (int m = 0; m < M; ++m)
        if ((rc = fill_model(kinds[m], prior_box + (size_t)m * VPET_PSTRIDE * 2, P.md[m])) != VPET_OK) return rc;
    if (o.proposal) {
        if (M != 1 || kinds[0] != KIND_IRR)
            return fail(VPET_E_MODEL, "the learned proposal drives the irreversible 2TCM alone");
        const int sl[4] = {VPET_SLOT_K1, VPET_SLOT_K2, VPET_SLOT_K3, VPET_SLOT_VB};
        const double share = o.proposal_prior_share, scale = o.proposal_sd_scale == 0.0 ? 1.0 : o.proposal_sd_scale;
        if (!(share >= 0.0 && share <= 1.0)) return fail(VPET_E_ARG, "opts.proposal_prior_share must lie in [0, 1]");
        if (!(std::isfinite(scale) && scale > 0.0)) return fail(VPET_E_ARG, "opts.proposal_sd_scale must be > 0");
        P.prop_logvol = 0.0;
        for (int j = 0; j < 4; ++j) {
            P.plo[j] = (float)prior_box[2 * sl[j]];
            P.phi[j] = (float)prior_box[2 * sl[j] + 1];
            P.prop_logvol += std::log((double)P.phi[j] - (double)P.plo[j]);
        }
        P.prop_share = share;
        P.prop_logscale = std::log(scale);
        P.prop = o.proposal;
        P.out_ess = o.out_ess;
    } else if (o.out_ess || o.accept_below) {
        return fail(VPET_E_ARG, "opts.out_ess and opts.accept_below need opts.proposal");
    }
    const double lambda = o.decay_lambda > 0.0 ? o.decay_lambda : std::log(2.0) / 109.8;
    HostTab T;
    if ((rc = make_tables(input_fn, frame_times, grid, lambda, T)) != VPET_OK) return rc;
    if (n_voxels == 0) return VPET_OK;
    if (!tacs || !out_moments || !out_model_prob)
        return fail(VPET_E_ARG, "tacs, out_moments and out_model_prob must not be NULL");

    const int cap = pow2_at_least((int)n_acc + 2 * kWave);
    int wpv = o.waves_per_voxel;
    if (wpv == 0) {
        wpv = 1;
        while (wpv < kMaxWpv && (double)n_voxels * wpv < 8192.0) wpv <<= 1;
    }
    auto lds_for = [&](int w) {
        return (size_t)((16 * T.F + 15) & ~15) + sizeof(uint64_t) * (size_t)w * cap + sizeof(double) * kRedStride * kMaxWpv + 16 +
               (o.proposal ? sizeof(MixTab) : 0);
    };
    while (wpv > 1 && lds_for(wpv) > (size_t)kLdsLimit) wpv >>= 1;
    if (lds_for(wpv) > (size_t)kLdsLimit) return fail(VPET_E_LIMIT, "selection buffer exceeds LDS");

    P.weights = o.weights;
    P.C0 = T.C0;
    P.h = T.h;
    P.floor_frac = o.weight_floor_frac > 0.0f ? (double)o.weight_floor_frac : 0.01;
    P.F = T.F;
    P.k0 = T.k0;
    P.M = M;
    P.cap = cap;
    P.wpv = wpv;
    P.l1 = o.distance;
    P.n_draws = (unsigned)n_draws;
    P.n_acc = (unsigned)n_acc;
    P.key0 = (unsigned)(seed & 0xffffffffu);
    P.key1 = (unsigned)(seed >> 32);
    P.out_mom = out_moments;
    P.out_prob = out_model_prob;
    P.out_idx = o.out_accept_idx;
    P.out_dist = o.out_accept_dist;
    P.out_thr = o.out_threshold;

    hipStream_t st = (hipStream_t)hip_stream;
    DevCtx* ctx = nullptr;
    std::unique_lock<std::mutex> lock;
    int slot = 0;
    if (noalloc) {
        if ((rc = stage_tables_noalloc(T, st, P.tab)) != VPET_OK) return rc;
    } else {
        if ((rc = current_ctx(&ctx)) != VPET_OK) return rc;
        lock = std::unique_lock<std::mutex>(ctx->mu);
        if ((rc = upload_tables(*ctx, T, st, P.tab, slot)) != VPET_OK) return rc;
    }
    const size_t lds = lds_for(wpv);
    const long long chunk = 1LL << 30;
    for (long long base = 0; base < n_voxels; base += chunk) {
        InferArgs Q = P;
        Q.V = std::min<long long>(n_voxels - base, chunk);
        Q.vbase = (unsigned long long)(o.voxel_offset + base);
        Q.tacs = tacs + (size_t)base * T.F;
        Q.weights = o.weights ? o.weights + (size_t)base * T.F : nullptr;
        Q.out_mom = out_moments + (size_t)base * M * 16;
        Q.out_prob = out_model_prob + (size_t)base * M;
        Q.out_idx = o.out_accept_idx ? o.out_accept_idx + (size_t)base * n_acc : nullptr;
        Q.out_dist = o.out_accept_dist ? o.out_accept_dist + (size_t)base * n_acc : nullptr;
        Q.out_thr = o.out_threshold ? o.out_threshold + base : nullptr;
        Q.prop = o.proposal ? o.proposal + (size_t)base * VPET_PROPOSAL_NOUT : nullptr;
        Q.out_ess = o.out_ess ? o.out_ess + base : nullptr;
        Q.below = o.accept_below ? o.accept_below + base : nullptr;
        const dim3 grid((unsigned)Q.V), block(kWave * wpv);
        const int sel = o.proposal ? -1 - o.distance : (M == 1 ? kinds[0] : 0) * 2 + (o.distance == 1 ? 1 : 0);
        switch (sel) {
            case -1: hipLaunchKernelGGL((vpet_infer_is_kernel<false>), grid, block, lds, st, Q); break;
            case -2: hipLaunchKernelGGL((vpet_infer_is_kernel<true>), grid, block, lds, st, Q); break;
            case 2 * KIND_IRR: hipLaunchKernelGGL((vpet_infer_kernel<KIND_IRR, false>), grid, block, lds, st, Q); break;
            case 2 * KIND_IRR + 1: hipLaunchKernelGGL((vpet_infer_kernel<KIND_IRR, true>), grid, block, lds, st, Q); break;
            case 2 * KIND_REV: hipLaunchKernelGGL((vpet_infer_kernel<KIND_REV, false>), grid, block, lds, st, Q); break;
            case 2 * KIND_REV + 1: hipLaunchKernelGGL((vpet_infer_kernel<KIND_REV, true>), grid, block, lds, st, Q); break;
            case 2 * KIND_1TCM: hipLaunchKernelGGL((vpet_infer_kernel<KIND_1TCM, false>), grid, block, lds, st, Q); break;
            case 2 * KIND_1TCM + 1: hipLaunchKernelGGL((vpet_infer_kernel<KIND_1TCM, true>), grid, block, lds, st, Q); break;
            case 1: hipLaunchKernelGGL((vpet_infer_kernel<0, true>), grid, block, lds, st, Q); break;
            default: hipLaunchKernelGGL((vpet_infer_kernel<0, false>), grid, block, lds, st, Q); break;
        }
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return hip_fail(e, "infer launch");
    }
    if (ctx) {
        hipError_t e = hipEventRecord(ctx->ev[slot], st);
        if (e != hipSuccess) return hip_fail(e, "hipEventRecord");
    }
    return VPET_OK;
}

int vpet_abc_infer(const float* tacs, int64_t n_voxels, const float* frame_times, const float* input_fn,
                   vpet_grid grid, uint32_t model_id, const double* prior_box, int64_t n_draws, double accept_frac,
                   uint64_t seed, float* out_moments, float* out_model_prob, const vpet_abc_opts* opts,
                   void* hip_stream) {
    return infer_entry(false, tacs, n_voxels, frame_times, input_fn, grid, model_id, prior_box, n_draws,
                       accept_frac, seed, out_moments, out_model_prob, opts, hip_stream);
}

int vpet_abc_infer_noalloc(const float* tacs, int64_t n_voxels, const float* frame_times, const float* input_fn,
                           vpet_grid grid, uint32_t model_id, const double* prior_box, int64_t n_draws,
                           double accept_frac, uint64_t seed, float* out_moments, float* out_model_prob,
                           const vpet_abc_opts* opts, void* hip_stream) {
    return infer_entry(true, tacs, n_voxels, frame_times, input_fn, grid, model_id, prior_box, n_draws,
                       accept_frac, seed, out_moments, out_model_prob, opts, hip_stream);
}

int vpet_abc_draws(uint32_t model_id, const double* prior_box, uint64_t seed, const int64_t* voxel,
                   const int64_t* draw, const int32_t* model_pos, int64_t count, uint32_t* out_words,
                   float* out_theta, void* hip_stream) {
    int kinds[kMaxModels];
    const int M = model_list(model_id, kinds);
    if (M < 1) return fail(VPET_E_MODEL, "unknown or empty model bitmask 0x%x", model_id);
    if (!prior_box) return fail(VPET_E_ARG, "prior_box must not be NULL");
    if (count < 0) return fail(VPET_E_ARG, "count must be >= 0");
    ModelDev md[kMaxModels] = {};
    int rc;
    for (int m = 0; m < M; ++m)
        if ((rc = fill_model(kinds[m], prior_box + (size_t)m * VPET_PSTRIDE * 2, md[m])) != VPET_OK) return rc;
    if (count == 0) return VPET_OK;
    if (!voxel || !draw || !model_pos || !out_words || !out_theta)
        return fail(VPET_E_ARG, "device pointers must not be NULL");
    hipStream_t st = (hipStream_t)hip_stream;
    const int threads = 256;
    for (long long base = 0; base < count; base += (1LL << 30)) {
        const long long cnt = std::min<long long>(count - base, 1LL << 30);
        hipLaunchKernelGGL(vpet_draws_kernel, dim3((unsigned)((cnt + threads - 1) / threads)), dim3(threads), 0, st,
                           md[0], md[1], md[2], M, (uint32_t)(seed & 0xffffffffu), (uint32_t)(seed >> 32),
                           voxel + base, draw + base, model_pos + base, cnt, out_words + (size_t)base * 8,
                           out_theta + (size_t)base * VPET_PSTRIDE);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return hip_fail(e, "draws launch");
    }
    return VPET_OK;
}


int vpet_abc_bank_ld(int32_t n_frames) { return n_frames <= 0 ? 0 : ((n_frames + 7) / 8) * 8; }

int vpet_abc_bank_build(uint32_t model_id, const double* prior_box, int64_t n_draws, uint64_t seed,
                        const float* input_fn, const float* frame_times, vpet_grid grid, float* out_theta,
                        double* out_x, void* hip_stream) {
    int kinds[kMaxModels];
    const int M = model_list(model_id, kinds);
    if (M < 1) return fail(VPET_E_MODEL, "unknown or empty model bitmask 0x%x", model_id);
    if (!prior_box) return fail(VPET_E_ARG, "prior_box must not be NULL");
    if (n_draws < 1) return fail(VPET_E_ARG, "n_draws must be >= 1");
    if ((double)M * (double)n_draws > 4294967295.0) return fail(VPET_E_LIMIT, "M * n_draws must stay below 2^32");
    ModelDev md[kMaxModels] = {};
    int rc;
    for (int m = 0; m < M; ++m)
        if ((rc = fill_model(kinds[m], prior_box + (size_t)m * VPET_PSTRIDE * 2, md[m])) != VPET_OK) return rc;
    HostTab T;
    if ((rc = make_tables(input_fn, frame_times, grid, 0.0, T)) != VPET_OK) return rc;
    if (T.F > VPET_BANK_MAX_FRAMES)
        return fail(VPET_E_LIMIT, "the bank form supports up to %d frames", VPET_BANK_MAX_FRAMES);
    if (!out_theta || !out_x) return fail(VPET_E_ARG, "out_theta and out_x must not be NULL");
    const int ld = vpet_abc_bank_ld(T.F);
    DevCtx* ctx;
    if ((rc = current_ctx(&ctx)) != VPET_OK) return rc;
    hipStream_t st = (hipStream_t)hip_stream;
    std::lock_guard<std::mutex> lock(ctx->mu);
    Tab tab;
    int slot;
    if ((rc = upload_tables(*ctx, T, st, tab, slot)) != VPET_OK) return rc;
    const unsigned threads = 256, blocks = (unsigned)((n_draws + threads - 1) / threads);
    const unsigned k0 = (unsigned)(seed & 0xffffffffu), k1 = (unsigned)(seed >> 32);
    for (int m = 0; m < M; ++m) {
#define VPET_BANK(KD)                                                                                  \
    hipLaunchKernelGGL(vpet_bank_kernel<KD>, dim3(blocks), dim3(threads), 0, st, md[m], m, (unsigned)n_draws, k0, \
                       k1, tab, T.C0, T.h, T.F, T.k0, ld, out_theta, out_x)
        switch (kinds[m]) {
            case KIND_1TCM: VPET_BANK(KIND_1TCM); break;
            case KIND_IRR: VPET_BANK(KIND_IRR); break;
            case KIND_REV: VPET_BANK(KIND_REV); break;
            case KIND_MRTM: VPET_BANK(KIND_MRTM); break;
            default: VPET_BANK(KIND_LPNT); break;
        }
#undef VPET_BANK
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return hip_fail(e, "bank launch");
    }
    hipError_t e = hipEventRecord(ctx->ev[slot], st);
    if (e != hipSuccess) return hip_fail(e, "hipEventRecord");
    return VPET_OK;
}

int vpet_abc_infer_bank(const float* tacs, int64_t n_voxels, const float* frame_times, vpet_grid grid,
                        uint32_t model_id, int64_t n_draws, double accept_frac, const float* bank_theta,
                        const double* bank_x, float* out_moments, float* out_model_prob, const vpet_abc_opts* opts,
                        void* hip_stream) {
    int kinds[kMaxModels];
    const int M = model_list(model_id, kinds);
    if (M < 1) return fail(VPET_E_MODEL, "unknown or empty model bitmask 0x%x", model_id);
    if (n_voxels < 0) return fail(VPET_E_ARG, "n_voxels must be >= 0");
    if (n_draws < 1) return fail(VPET_E_ARG, "n_draws must be >= 1");
    if ((double)M * (double)n_draws > 4294967295.0) return fail(VPET_E_LIMIT, "M * n_draws must stay below 2^32");
    vpet_abc_opts o{};
    if (opts) o = *opts;
    if (o.distance != 0 && o.distance != 1) return fail(VPET_E_ARG, "opts.distance must be 0 (L2) or 1 (L1)");
    if (!(std::isfinite(o.decay_lambda) && o.decay_lambda >= 0.0))
        return fail(VPET_E_ARG, "opts.decay_lambda must be finite and >= 0");
    if (!(std::isfinite(o.weight_floor_frac) && o.weight_floor_frac >= 0.0f))
        return fail(VPET_E_ARG, "opts.weight_floor_frac must be finite and >= 0");
    if (o.bank_pilot < 0) return fail(VPET_E_ARG, "opts.bank_pilot must be >= 0");
    if (o.bank_scan < 0 || o.bank_scan > 2) return fail(VPET_E_ARG, "opts.bank_scan must be 0, 1 or 2");
    if (o.bank_scan == 2 && o.distance == 1)
        return fail(VPET_E_ARG, "the bf16 contraction scan needs the L2 distance");
    if (o.proposal || o.out_ess || o.accept_below)
        return fail(VPET_E_ARG, "opts.proposal, opts.out_ess and opts.accept_below do not apply to a prior bank");
    const bool use_mfma = o.bank_scan == 2 || (o.bank_scan == 0 && o.distance == 0);
    int64_t n_acc = 0;
    int rc = vpet_abc_accept_count((int64_t)M * n_draws, accept_frac, &n_acc);
    if (rc != VPET_OK) return rc;
    if (n_acc > VPET_BANK_MAX_ACCEPT)
        return fail(VPET_E_LIMIT, "n = %lld exceeds VPET_BANK_MAX_ACCEPT = %d", (long long)n_acc,
                    VPET_BANK_MAX_ACCEPT);
    // frame bounds and weights' decay factors (the input function is not needed)
    const int F = grid.n_frames;
    std::vector<double> omega;
    if ((rc = bank_omega(frame_times, grid, o.decay_lambda, omega)) != VPET_OK) return rc;
    if (n_voxels == 0) return VPET_OK;
    if (!tacs || !out_moments || !out_model_prob || !bank_theta || !bank_x)
        return fail(VPET_E_ARG, "tacs, bank and output pointers must not be NULL");
    const int64_t n_tot = (int64_t)M * n_draws;
    // candidate buffer per voxel: the contraction's error margin admits rows
    // somewhat above the threshold, so it gets twice the room (up to 4096)
    const int cap = use_mfma ? std::max(512, std::min(4096, pow2_at_least(16 * (int)n_acc)))
                             : std::max(256, pow2_at_least(8 * (int)n_acc));
    const size_t cand_bytes = sizeof(uint64_t);  // (fp32 distance or computed S, bank row)
    // default pilot: about 4 n bank rows below the threshold (FP64 scan: the
    // 16th smallest of 4 N / n rows; contraction scan: the 16th smallest of 32
    // column minima over 5.5 N / n rows)
    int64_t pilot = o.bank_pilot > 0 ? o.bank_pilot
                    : use_mfma       ? (11 * n_tot + 2 * n_acc - 1) / (2 * n_acc)
                                     : (4 * n_tot + n_acc - 1) / n_acc;
    pilot = std::min<int64_t>(pilot, n_tot);
    const int ld = vpet_abc_bank_ld(F);

    BankArgs A{};
    A.weights = o.weights;
    A.bank_x = bank_x;
    A.bank_theta = bank_theta;
    A.floor_frac = o.weight_floor_frac > 0.0f ? (double)o.weight_floor_frac : 0.01;
    A.F = F;
    A.ld = ld;
    A.l1 = o.distance;
    A.M = M;
    A.cap = cap;
    A.n_tot = (unsigned)n_tot;
    A.n_draws = (unsigned)n_draws;
    A.n_acc = (unsigned)n_acc;
    A.n_pilot = (unsigned)pilot;
    for (int m = 0; m < M; ++m) A.kinds[m] = kinds[m];

    DevCtx* ctx;
    if ((rc = current_ctx(&ctx)) != VPET_OK) return rc;
    hipStream_t st = (hipStream_t)hip_stream;
    std::lock_guard<std::mutex> lock(ctx->mu);
    int slot;
    const void* dom;
    if ((rc = upload_blob(*ctx, omega.data(), sizeof(double) * F, st, &dom, slot)) != VPET_OK) return rc;
    A.omega = static_cast<const double*>(dom);

    // voxel chunks bound the candidate work to ~4 GiB
    const long long chunk = std::max<long long>(256, (1LL << 32) / ((long long)cap * (long long)cand_bytes));
    const long long cv = std::min<long long>(n_voxels, chunk);
    const int KB = 2 * ld;  // contraction length: [x, x^2] per frame
    char* work = nullptr;
    const size_t sz_tau = align256(sizeof(float) * cv), sz_cnt = align256(sizeof(int) * 2 * cv);
    const size_t sz_fb = align256(sizeof(int) * cv) + 256, sz_cand = align256(cand_bytes * (size_t)cap * cv);
    const size_t sz_b = use_mfma ? align256(sizeof(uint16_t) * (size_t)KB * n_tot) : 0;
    const size_t sz_a = use_mfma ? align256(sizeof(uint16_t) * (size_t)KB * cv) : 0;
    const size_t sz_c = use_mfma ? align256(sizeof(float) * cv) : 0;
    const size_t sz_av = use_mfma ? align256(sizeof(double) * cv) : 0;
    hipError_t e = hipMallocAsync((void**)&work, sz_tau + sz_cnt + sz_fb + sz_cand + 2 * sz_b + 2 * sz_a + 3 * sz_c + sz_av, st);
    if (e != hipSuccess) return fail(VPET_E_NOMEM, "bank work: %s", hipGetErrorString(e));
    char* q = work;
    A.tau = reinterpret_cast<float*>(q);
    q += sz_tau;
    A.cnt = reinterpret_cast<int*>(q);
    A.cnt_hi = A.cnt + cv;
    q += sz_cnt;
    A.fb_count = reinterpret_cast<unsigned*>(q);
    A.fb_list = reinterpret_cast<int*>(q + 256);
    q += sz_fb;
    A.cand = reinterpret_cast<uint64_t*>(q);
    q += sz_cand;
    A.K = KB;
    if (use_mfma) {
        A.bhi = reinterpret_cast<uint16_t*>(q);
        q += sz_b;
        A.blo = reinterpret_cast<uint16_t*>(q);
        q += sz_b;
        A.ahi = reinterpret_cast<uint16_t*>(q);
        q += sz_a;
        A.alo = reinterpret_cast<uint16_t*>(q);
        q += sz_a;
        A.cthr = reinterpret_cast<float*>(q);
        q += sz_c;
        A.cthr1 = reinterpret_cast<float*>(q);
        q += sz_c;
        A.tau1 = reinterpret_cast<float*>(q);
        q += sz_c;
        A.aval = reinterpret_cast<double*>(q);
    }
    A.scap = select_key_buffer(cap, (int)n_acc, false);
    const size_t lds = sizeof(uint64_t) * (use_mfma ? A.scap : cap) + sizeof(double) * kRedStride * kMaxWpv +
                       (use_mfma ? 2 * sizeof(double) * (size_t)ld + sizeof(uint32_t) * 2 * kWave : 0);
    // fallback blocks: up to 8 wavefronts, each with its own pow2(n + 128)-key
    // top-n, within 48 KB of LDS
    const int fb_cap = pow2_at_least((int)n_acc + 2 * kWave);
    int fb_waves = 8;
    while (fb_waves > 1 && (size_t)fb_waves * fb_cap * sizeof(uint64_t) > 48 * 1024) fb_waves >>= 1;
    const size_t fb_lds = sizeof(uint64_t) * (size_t)fb_waves * fb_cap + sizeof(double) * kRedStride * fb_waves;
    A.fb_cap = fb_cap;
    const bool mfma = use_mfma;
    if (o.out_fallback_voxels) *o.out_fallback_voxels = 0;
    hipEvent_t tev[2] = {nullptr, nullptr};  // brackets the scan kernel of each chunk
    if (o.out_scan_ms) {
        *o.out_scan_ms = 0.0f;
        for (hipEvent_t& ev : tev) {
            e = hipEventCreate(&ev);
            if (e != hipSuccess) rc = hip_fail(e, "hipEventCreate");
        }
    }
    auto mark = [&](int k) {
        if (!tev[k]) return;
        const hipError_t me = hipEventRecord(tev[k], st);
        if (me != hipSuccess && rc == VPET_OK) rc = hip_fail(me, "hipEventRecord");
    };
    if (mfma) {
        bank_bops(A, (unsigned)n_tot, st, ld);
        e = hipGetLastError();
        if (e != hipSuccess) rc = hip_fail(e, "bank operand launch");
    }
    for (long long base = 0; base < n_voxels && rc == VPET_OK; base += cv) {
        BankArgs Q = A;
        Q.V = std::min<long long>(n_voxels - base, cv);
        Q.tacs = tacs + (size_t)base * F;
        Q.weights = o.weights ? o.weights + (size_t)base * F : nullptr;
        Q.out_mom = out_moments + (size_t)base * M * 16;
        Q.out_prob = out_model_prob + (size_t)base * M;
        Q.out_idx = o.out_accept_idx ? o.out_accept_idx + (size_t)base * n_acc : nullptr;
        Q.out_dist = o.out_accept_dist ? o.out_accept_dist + (size_t)base * n_acc : nullptr;
        Q.out_thr = o.out_threshold ? o.out_threshold + base : nullptr;
        bank_chunk(Q, st, ld, o.distance == 1, mfma, lds, fb_lds, fb_waves, mark);
        e = hipGetLastError();
        if (e != hipSuccess) rc = hip_fail(e, "bank infer launch");
        if (o.out_fallback_voxels && rc == VPET_OK) {
            unsigned nfb = 0;
            e = hipMemcpyAsync(&nfb, Q.fb_count, sizeof nfb, hipMemcpyDeviceToHost, st);
            if (e == hipSuccess) e = hipStreamSynchronize(st);
            if (e != hipSuccess) rc = hip_fail(e, "fallback count");
            *o.out_fallback_voxels += nfb;
        }
        if (tev[0] && rc == VPET_OK) {
            e = hipEventSynchronize(tev[1]);
            float ms = 0.0f;
            if (e == hipSuccess) e = hipEventElapsedTime(&ms, tev[0], tev[1]);
            if (e != hipSuccess) rc = hip_fail(e, "scan timing");
            *o.out_scan_ms += ms;
        }
    }
    for (hipEvent_t ev : tev)
        if (ev) (void)hipEventDestroy(ev);  // after the waits above: nothing pending
    e = hipFreeAsync(work, st);
    if (e != hipSuccess && rc == VPET_OK) rc = hip_fail(e, "hipFreeAsync");
    e = hipEventRecord(ctx->ev[slot], st);
    if (e != hipSuccess && rc == VPET_OK) rc = hip_fail(e, "hipEventRecord");
    return rc;
}


int vpet_abc_infer_bank_learned(const float* tacs, int64_t n_voxels, const float* frame_times, const float* input_fn,
                                vpet_grid grid, uint32_t model_id, const double* prior_box, const float* proposal,
                                const vpet_bank_groups* groups, int64_t n_draws, double accept_frac, uint64_t seed,
                                float* out_moments, float* out_model_prob, const vpet_abc_opts* opts,
                                void* hip_stream) {
    int kinds[kMaxModels];
    const int M = model_list(model_id, kinds);
    if (M < 1 || (model_id & ~(uint32_t)(VPET_M_2TCM_IRR | VPET_M_2TCM_REV)) != 0u)
        return fail(VPET_E_MODEL, "the learned bank runs the irreversible and reversible 2TCM (model_id 0x%x)", model_id);
    if (n_voxels < 0) return fail(VPET_E_ARG, "n_voxels must be >= 0");
    if (!prior_box || !groups) return fail(VPET_E_ARG, "prior_box and groups must not be NULL");
    if (n_draws < 1) return fail(VPET_E_ARG, "n_draws must be >= 1");
    const vpet_bank_groups gp = *groups;
    if (gp.dims != 4 && gp.dims != 5) return fail(VPET_E_ARG, "groups->dims must be 4 or 5");
    if (gp.bins < 1) return fail(VPET_E_ARG, "groups->bins must be >= 1");
    double ncell_d = 1.0;
    for (int j = 0; j < gp.dims; ++j) ncell_d *= gp.bins;
    if (ncell_d > kLbMaxCells) return fail(VPET_E_LIMIT, "bins^dims must not exceed %d", kLbMaxCells);
    if (gp.group_voxels < kLbVox || gp.group_voxels % kLbVox != 0)
        return fail(VPET_E_ARG, "groups->group_voxels must be a positive multiple of %d", kLbVox);
    if (!(gp.prior_share >= 0.0 && gp.prior_share <= 1.0)) return fail(VPET_E_ARG, "groups->prior_share must lie in [0, 1]");
    const double scale = gp.sd_scale == 0.0 ? 1.0 : gp.sd_scale;
    if (!(std::isfinite(scale) && scale > 0.0)) return fail(VPET_E_ARG, "groups->sd_scale must be > 0");
    if (gp.first_group < 0 || (double)gp.first_group + (double)n_voxels / gp.group_voxels + 1.0 > 4294967296.0)
        return fail(VPET_E_ARG, "group indices (first_group + g) must lie in [0, 2^32)");
    vpet_abc_opts o{};
    if (opts) o = *opts;
    if (o.proposal || o.waves_per_voxel != 0 || o.voxel_offset != 0)
        return fail(VPET_E_ARG, "opts.proposal, waves_per_voxel and voxel_offset do not apply to the learned bank");
    if (o.distance != 0 && o.distance != 1) return fail(VPET_E_ARG, "opts.distance must be 0 (L2) or 1 (L1)");
    if (!(std::isfinite(o.decay_lambda) && o.decay_lambda >= 0.0))
        return fail(VPET_E_ARG, "opts.decay_lambda must be finite and >= 0");
    if (!(std::isfinite(o.weight_floor_frac) && o.weight_floor_frac >= 0.0f))
        return fail(VPET_E_ARG, "opts.weight_floor_frac must be finite and >= 0");
    if (o.bank_pilot < 0) return fail(VPET_E_ARG, "opts.bank_pilot must be >= 0");
    if (o.bank_scan < 0 || o.bank_scan > 2) return fail(VPET_E_ARG, "opts.bank_scan must be 0, 1 or 2");
    if (o.bank_scan == 2 && o.distance == 1) return fail(VPET_E_ARG, "the bf16 contraction scan needs the L2 distance");
    const bool mfma = o.bank_scan == 2 || (o.bank_scan == 0 && o.distance == 0);
    if ((double)M * (double)n_draws > 4294967295.0) return fail(VPET_E_LIMIT, "M * n_draws must stay below 2^32");
    const int64_t n_tot = (int64_t)M * n_draws;  // bank rows per group
    int64_t n_acc = 0;
    int rc = vpet_abc_accept_count(n_tot, accept_frac, &n_acc);
    if (rc != VPET_OK) return rc;
    if (n_acc > VPET_BANK_MAX_ACCEPT)
        return fail(VPET_E_LIMIT, "n = %lld exceeds VPET_BANK_MAX_ACCEPT = %d", (long long)n_acc, VPET_BANK_MAX_ACCEPT);
    ModelDev md[kMaxModels] = {};
    for (int m = 0; m < M; ++m)
        if ((rc = fill_model(kinds[m], prior_box + (size_t)m * VPET_PSTRIDE * 2, md[m])) != VPET_OK) return rc;
    const double lambda = o.decay_lambda > 0.0 ? o.decay_lambda : std::log(2.0) / 109.8;
    HostTab T;
    if ((rc = make_tables(input_fn, frame_times, grid, lambda, T)) != VPET_OK) return rc;
    const int F = T.F;
    if (F > VPET_BANK_MAX_FRAMES) return fail(VPET_E_LIMIT, "the bank form supports up to %d frames", VPET_BANK_MAX_FRAMES);
    std::vector<double> omega;
    if ((rc = bank_omega(frame_times, grid, o.decay_lambda, omega)) != VPET_OK) return rc;
    if (n_voxels == 0) return VPET_OK;
    if (!tacs || !proposal || !out_moments || !out_model_prob)
        return fail(VPET_E_ARG, "tacs, proposal and output pointers must not be NULL");
    if (n_voxels > (int64_t)INT32_MAX) return fail(VPET_E_LIMIT, "at most 2^31 - 1 voxels per call");

    // the head parameter of each model parameter (draw order K1, k2, k3, [k4,] vB)
    LbBank LB{};
    const int S = gp.group_voxels;
    const int64_t G = (n_voxels + S - 1) / S;
    const int ld = vpet_abc_bank_ld(F);
    const int KB = 2 * ld;
    // device scratch of the grouping (whole call) and of one voxel chunk; a
    // chunk holds whole groups, its candidate list stays within 4 GiB and its
    // banks within 16 GiB (large banks of many groups would otherwise cut the
    // chunks below the size that fills the chip)
    const int cap = mfma ? std::max(512, std::min(4096, pow2_at_least(16 * (int)n_acc)))
                         : std::max(256, pow2_at_least(8 * (int)n_acc));
    const size_t row_bytes = sizeof(float) * VPET_PSTRIDE + sizeof(double) * (size_t)ld + sizeof(double) +
                             (mfma ? 2 * sizeof(uint16_t) * (size_t)KB : 0);
    long long cv = std::max<long long>(S, (1LL << 32) / ((long long)cap * (long long)sizeof(uint64_t)));
    cv = std::max<long long>(S, std::min<long long>(cv, (long long)((1ULL << 34) / (row_bytes * (size_t)n_tot)) * S));
    cv = std::max<long long>(S, (cv / S) * S);
    cv = std::min<long long>(cv, ((n_voxels + S - 1) / S) * S);
    const long long gpc = cv / S;  // groups per chunk
    if ((double)gpc * (double)n_tot > 4294967295.0) return fail(VPET_E_LIMIT, "groups x bank rows must stay below 2^32");
    const int D = gp.dims;
    const int ncell = (int)ncell_d;
    const long long V = n_voxels;
    const int nb = (int)((V + kLbBlock - 1) / kLbBlock);
    auto a256 = [](size_t b) { return align256(b); };
    const size_t sz_key = a256(sizeof(unsigned) * V), sz_zm = a256(sizeof(double) * 2 * D * V),
                 sz_hist = a256(sizeof(int) * (size_t)nb * (ncell + 1)), sz_perm = a256(sizeof(int) * V),
                 sz_ys = a256(sizeof(float) * (size_t)F * V), sz_ws = o.weights ? sz_ys : 0,
                 sz_grp = a256(sizeof(LbGroup) * G), sz_tot = a256(sizeof(int) * (ncell + 1)),
                 sz_ref = mfma ? a256(sizeof(double) * (size_t)ld * G) : 0;
    const size_t rows_c = (size_t)gpc * n_tot;
    const size_t sz_bt = gp.out_bank_theta ? 0 : a256(sizeof(float) * VPET_PSTRIDE * rows_c),
                 sz_bx = a256(sizeof(double) * (size_t)ld * rows_c),
                 sz_bw = gp.out_bank_logw ? 0 : a256(sizeof(double) * rows_c),
                 sz_b = mfma ? a256(sizeof(uint16_t) * (size_t)KB * rows_c) : 0;
    const size_t sz_tau = a256(sizeof(float) * cv), sz_cnt = a256(sizeof(int) * 2 * cv),
                 sz_fb = a256(sizeof(int) * cv) + 256, sz_cand = a256(sizeof(uint64_t) * (size_t)cap * cv),
                 sz_a = mfma ? a256(sizeof(uint16_t) * (size_t)KB * cv) : 0, sz_c = mfma ? a256(sizeof(float) * cv) : 0,
                 sz_av = mfma ? a256(sizeof(double) * cv) : 0;
    const size_t total = sz_key + sz_zm + sz_hist + sz_perm + sz_ys + sz_ws + sz_grp + sz_tot + sz_ref + sz_bt + sz_bx +
                         sz_bw +
                         2 * sz_b + sz_tau + sz_cnt + sz_fb + sz_cand + 2 * sz_a + 3 * sz_c + sz_av;

    DevCtx* ctx;
    if ((rc = current_ctx(&ctx)) != VPET_OK) return rc;
    hipStream_t st = (hipStream_t)hip_stream;
    std::lock_guard<std::mutex> lock(ctx->mu);
    int slot;
    Tab tab;
    if ((rc = upload_tables(*ctx, T, st, tab, slot)) != VPET_OK) return rc;
    // the weights' decay factors sit in the same slot, after the tables
    const size_t off_om = align256(tab_layout(T).bytes);
    if (off_om + sizeof(double) * F > kSlotBytes) {
        (void)hipEventRecord(ctx->ev[slot], st);
        return fail(VPET_E_LIMIT, "tables exceed a slot");
    }
    std::memcpy(ctx->hbuf + (size_t)slot * kSlotBytes + off_om, omega.data(), sizeof(double) * F);
    double* d_omega = reinterpret_cast<double*>(ctx->dbuf + (size_t)slot * kSlotBytes + off_om);
    hipError_t e = hipMemcpyAsync(d_omega, ctx->hbuf + (size_t)slot * kSlotBytes + off_om, sizeof(double) * F,
                                  hipMemcpyHostToDevice, st);
    if (e != hipSuccess) return hip_fail(e, "omega upload");
    char* work = nullptr;
    e = hipMallocAsync((void**)&work, total, st);
    if (e != hipSuccess) {
        (void)hipEventRecord(ctx->ev[slot], st);
        return fail(VPET_E_NOMEM, "learned bank work: %s", hipGetErrorString(e));
    }
    char* q = work;
    auto carve = [&](size_t b) {
        char* r = q;
        q += b;
        return r;
    };
    LbArgs A{};
    A.prop = proposal;
    A.tacs = tacs;
    A.weights = o.weights;
    A.V = V;
    A.F = F;
    A.D = D;
    A.bins = gp.bins;
    A.ncell = ncell;
    A.nb = nb;
    A.S = S;
    A.out_group = gp.out_group;
    {
        // cells over the box of the head's parameters (K1, k2, k3, [k4,] vB) of
        // the last model listed (the reversible one when both are)
        const double* box = prior_box + (size_t)(M - 1) * VPET_PSTRIDE * 2;
        const int hs4[4] = {VPET_SLOT_K1, VPET_SLOT_K2, VPET_SLOT_K3, VPET_SLOT_VB};
        const int hs5[5] = {VPET_SLOT_K1, VPET_SLOT_K2, VPET_SLOT_K3, VPET_SLOT_K4, VPET_SLOT_VB};
        for (int j = 0; j < D; ++j) {
            const int sl = D == 4 ? hs4[j] : hs5[j];
            A.clo[j] = (float)box[2 * sl];
            A.cwid[j] = (float)(box[2 * sl + 1] - box[2 * sl]);
            if (!(A.cwid[j] > 0.0f)) A.cwid[j] = 1.0f;  // a fixed parameter: one cell
        }
    }
    A.key = reinterpret_cast<unsigned*>(carve(sz_key));
    A.zmom = reinterpret_cast<double*>(carve(sz_zm));
    A.hist = reinterpret_cast<int*>(carve(sz_hist));
    A.perm = reinterpret_cast<int*>(carve(sz_perm));
    A.ys = reinterpret_cast<float*>(carve(sz_ys));
    A.ws = o.weights ? reinterpret_cast<float*>(carve(sz_ws)) : nullptr;
    LbGroup* d_groups = reinterpret_cast<LbGroup*>(carve(sz_grp));
    int* d_tot = reinterpret_cast<int*>(carve(sz_tot));
    double* d_ref = mfma ? reinterpret_cast<double*>(carve(sz_ref)) : nullptr;
    float* b_theta = gp.out_bank_theta ? nullptr : reinterpret_cast<float*>(carve(sz_bt));
    double* b_x = reinterpret_cast<double*>(carve(sz_bx));
    double* b_logw = gp.out_bank_logw ? nullptr : reinterpret_cast<double*>(carve(sz_bw));

    BankArgs B{};
    B.weights = A.ws;
    B.omega = d_omega;
    B.bank_x = b_x;
    B.floor_frac = o.weight_floor_frac > 0.0f ? (double)o.weight_floor_frac : 0.01;
    B.F = F;
    B.ld = ld;
    B.l1 = o.distance;
    B.M = M;
    B.cap = cap;
    B.n_tot = (unsigned)n_tot;
    B.n_draws = (unsigned)n_draws;
    B.n_acc = (unsigned)n_acc;
    int64_t pilot = o.bank_pilot > 0 ? o.bank_pilot
                    : mfma           ? (11 * n_tot + 2 * n_acc - 1) / (2 * n_acc)
                                     : (4 * n_tot + n_acc - 1) / n_acc;
    B.n_pilot = (unsigned)std::min<int64_t>(pilot, n_tot);
    for (int m = 0; m < M; ++m) B.kinds[m] = kinds[m];
    B.K = KB;
    if (mfma) {
        B.bhi = reinterpret_cast<uint16_t*>(carve(sz_b));
        B.blo = reinterpret_cast<uint16_t*>(carve(sz_b));
    }
    B.tau = reinterpret_cast<float*>(carve(sz_tau));
    B.cnt = reinterpret_cast<int*>(carve(sz_cnt));
    B.cnt_hi = B.cnt + cv;
    {
        char* fb = carve(sz_fb);
        B.fb_count = reinterpret_cast<unsigned*>(fb);
        B.fb_list = reinterpret_cast<int*>(fb + 256);
    }
    B.cand = reinterpret_cast<uint64_t*>(carve(sz_cand));
    if (mfma) {
        B.ahi = reinterpret_cast<uint16_t*>(carve(sz_a));
        B.alo = reinterpret_cast<uint16_t*>(carve(sz_a));
        B.cthr = reinterpret_cast<float*>(carve(sz_c));
        B.cthr1 = reinterpret_cast<float*>(carve(sz_c));
        B.tau1 = reinterpret_cast<float*>(carve(sz_c));
        B.aval = reinterpret_cast<double*>(carve(sz_av));
    }
    B.grp_vox = (unsigned)S;
    B.grp_rows = (unsigned)n_tot;
    B.out_row = A.perm;
    B.out_mom = out_moments;
    B.out_prob = out_model_prob;
    B.out_idx = o.out_accept_idx;
    B.out_dist = o.out_accept_dist;
    B.out_thr = o.out_threshold;
    B.out_ess = o.out_ess;
    B.below = o.accept_below;

    LB.groups = d_groups;
    LB.D = D;
    LB.share = gp.prior_share;
    LB.log_share = std::log(gp.prior_share);
    LB.log_rest = std::log1p(-gp.prior_share);
    LB.n_draws = (unsigned)n_draws;
    LB.rows_per_group = (unsigned)n_tot;
    LB.key0 = (unsigned)(seed & 0xffffffffu);
    LB.key1 = (unsigned)(seed >> 32);
    LB.ld = ld;
    LB.first = gp.first_group;

    // grouping: cells, stable order, groups and their Gaussians
    const dim3 b256(256);
    hipLaunchKernelGGL(vpet_lb_summary_kernel, dim3((unsigned)((V + 255) / 256)), b256, 0, st, A);
    hipLaunchKernelGGL(vpet_lb_hist_kernel, dim3((unsigned)nb), b256, 0, st, A);
    hipLaunchKernelGGL(vpet_lb_columns_kernel, dim3((unsigned)((ncell + 1 + 255) / 256)), b256, 0, st, A, d_tot);
    hipLaunchKernelGGL(vpet_lb_cellbase_kernel, dim3(1), dim3(1024), 0, st, A, d_tot);
    hipLaunchKernelGGL(vpet_lb_scatter_kernel, dim3((unsigned)nb), dim3(64), 0, st, A, (const int*)d_tot);
    hipLaunchKernelGGL(vpet_lb_gather_kernel, dim3((unsigned)((V * F + 255) / 256)), b256, 0, st, A);
    hipLaunchKernelGGL(vpet_lb_fit_kernel, dim3((unsigned)G), b256, 0, st, A, d_groups, scale);
    if (mfma) hipLaunchKernelGGL(vpet_lb_ref_kernel, dim3((unsigned)G), b256, 0, st, A, d_ref, ld);
    e = hipGetLastError();
    if (e != hipSuccess) rc = hip_fail(e, "grouping launch");

    // the re-ranking select keeps at most 8 n keys at or below tau in LDS
    // (about 4 n are expected; more go to the exact fallback)
    B.scap = select_key_buffer(cap, (int)n_acc, true);
    // (n <= VPET_BANK_MAX_ACCEPT = 512 makes this pow2(8 n) >= 8 n: the
    // weighted select stages 5 n values past the n accepted keys)
    const size_t lds = sizeof(uint64_t) * (mfma ? B.scap : cap) + sizeof(double) * kRedStride * kMaxWpv +
                       (mfma ? 2 * sizeof(double) * (size_t)ld + sizeof(uint32_t) * 2 * kWave : 0);
    const int fb_cap = pow2_at_least((int)n_acc + 2 * kWave);
    int fb_waves = 8;
    while (fb_waves > 1 && (size_t)fb_waves * fb_cap * sizeof(uint64_t) > 48 * 1024) fb_waves >>= 1;
    const size_t fb_lds = sizeof(uint64_t) * (size_t)fb_waves * fb_cap + sizeof(double) * kRedStride * fb_waves;
    B.fb_cap = fb_cap;
    if (o.out_fallback_voxels) *o.out_fallback_voxels = 0;
    hipEvent_t tev[2] = {nullptr, nullptr};
    if (o.out_scan_ms) {
        *o.out_scan_ms = 0.0f;
        for (hipEvent_t& ev : tev) {
            e = hipEventCreate(&ev);
            if (e != hipSuccess && rc == VPET_OK) rc = hip_fail(e, "hipEventCreate");
        }
    }
    auto mark = [&](int k) {
        if (!tev[k]) return;
        const hipError_t me = hipEventRecord(tev[k], st);
        if (me != hipSuccess && rc == VPET_OK) rc = hip_fail(me, "hipEventRecord");
    };
    for (long long base = 0; base < V && rc == VPET_OK; base += cv) {
        const long long nv = std::min<long long>(V - base, cv);
        const long long g0 = base / S, ng = (nv + S - 1) / S;
        // the chunk's banks
        LB.g0 = g0;
        LB.theta = gp.out_bank_theta ? gp.out_bank_theta + (size_t)g0 * n_tot * VPET_PSTRIDE : b_theta;
        LB.logw = gp.out_bank_logw ? gp.out_bank_logw + (size_t)g0 * n_tot : b_logw;
        LB.x = b_x;
        // with the contraction screen the bank kernel also writes the rows'
        // BF16 operands (bank_bops' output) from its staged curves
        LB.bhi = mfma ? B.bhi : nullptr;
        LB.blo = mfma ? B.blo : nullptr;
        LB.ref = d_ref ? d_ref + (size_t)g0 * ld : nullptr;
        for (int m = 0; m < M; ++m) {
            for (int p = 0; p < kMaxParams; ++p) LB.dim_of[p] = -1;
            // draw order K1, k2, k3, vB (irreversible) or K1, k2, k3, k4, vB
            LB.dim_of[0] = 0;
            LB.dim_of[1] = 1;
            LB.dim_of[2] = 2;
            if (kinds[m] == KIND_IRR) {
                LB.dim_of[3] = D - 1;
            } else {
                LB.dim_of[3] = D == 5 ? 3 : -1;
                LB.dim_of[4] = D - 1;
            }
            // a wavefront per 64 rows, its curves staged in LDS
            const dim3 bg((unsigned)((n_draws + kWave - 1) / kWave), (unsigned)ng), bw(kWave);
            const size_t stage = sizeof(double) * ((size_t)kWave * (ld + 1) + ld);
            if (kinds[m] == KIND_IRR)
                hipLaunchKernelGGL(vpet_lb_bank_kernel<KIND_IRR>, bg, bw, stage, st, LB, md[m], m, tab, T.C0, T.h, F,
                                   T.k0);
            else
                hipLaunchKernelGGL(vpet_lb_bank_kernel<KIND_REV>, bg, bw, stage, st, LB, md[m], m, tab, T.C0, T.h, F,
                                   T.k0);
        }
        BankArgs Q = B;
        Q.bank_theta = LB.theta;
        Q.bank_logw = LB.logw;
        Q.ref = d_ref ? d_ref + (size_t)g0 * ld : nullptr;
        Q.V = nv;
        Q.pos0 = base;
        Q.g0 = g0;
        Q.tacs = A.ys + (size_t)base * F;
        Q.weights = A.ws ? A.ws + (size_t)base * F : nullptr;
        bank_chunk(Q, st, ld, o.distance == 1, mfma, lds, fb_lds, fb_waves, mark);
        e = hipGetLastError();
        if (e != hipSuccess) rc = hip_fail(e, "learned bank launch");
        if (o.out_fallback_voxels && rc == VPET_OK) {
            unsigned nfb = 0;
            e = hipMemcpyAsync(&nfb, Q.fb_count, sizeof nfb, hipMemcpyDeviceToHost, st);
            if (e == hipSuccess) e = hipStreamSynchronize(st);
            if (e != hipSuccess) rc = hip_fail(e, "fallback count");
            *o.out_fallback_voxels += nfb;
        }
        if (tev[0] && rc == VPET_OK) {
            e = hipEventSynchronize(tev[1]);
            float ms = 0.0f;
            if (e == hipSuccess) e = hipEventElapsedTime(&ms, tev[0], tev[1]);
            if (e != hipSuccess) rc = hip_fail(e, "scan timing");
            *o.out_scan_ms += ms;
        }
    }
    for (hipEvent_t ev : tev)
        if (ev) (void)hipEventDestroy(ev);
    e = hipFreeAsync(work, st);
    if (e != hipSuccess && rc == VPET_OK) rc = hip_fail(e, "hipFreeAsync");
    e = hipEventRecord(ctx->ev[slot], st);
    if (e != hipSuccess && rc == VPET_OK) rc = hip_fail(e, "hipEventRecord");
    return rc;
}


int vpet_abc_bank_screen(const float* tacs, int64_t n_voxels, const float* frame_times, vpet_grid grid,
                         const double* bank_x, int64_t n_rows, const vpet_abc_opts* opts, float* out_s,
                         double* out_a, void* hip_stream) {
    if (n_voxels < 0) return fail(VPET_E_ARG, "n_voxels must be >= 0");
    if (n_voxels > kScreenMaxVoxels)
        return fail(VPET_E_LIMIT, "bank_screen takes at most %d voxels", kScreenMaxVoxels);
    if (n_rows < 1) return fail(VPET_E_ARG, "n_rows must be >= 1");
    if (n_rows > kScreenMaxRows) return fail(VPET_E_LIMIT, "bank_screen takes at most %d bank rows", kScreenMaxRows);
    vpet_abc_opts o{};
    if (opts) o = *opts;
    if (!(std::isfinite(o.decay_lambda) && o.decay_lambda >= 0.0))
        return fail(VPET_E_ARG, "opts.decay_lambda must be finite and >= 0");
    if (!(std::isfinite(o.weight_floor_frac) && o.weight_floor_frac >= 0.0f))
        return fail(VPET_E_ARG, "opts.weight_floor_frac must be finite and >= 0");
    std::vector<double> omega;
    int rc = bank_omega(frame_times, grid, o.decay_lambda, omega);
    if (rc != VPET_OK) return rc;
    if (n_voxels == 0) return VPET_OK;
    if (!tacs || !bank_x || !out_s || !out_a) return fail(VPET_E_ARG, "device pointers must not be NULL");
    const int F = grid.n_frames, ld = vpet_abc_bank_ld(F), KB = 2 * ld;
    // each half of a list can hold every row (the contraction scan fills both)
    const int cap = 2 * pow2_at_least((int)n_rows);
    BankArgs A{};
    A.tacs = tacs;
    A.weights = o.weights;
    A.bank_x = bank_x;
    A.floor_frac = o.weight_floor_frac > 0.0f ? (double)o.weight_floor_frac : 0.01;
    A.F = F;
    A.ld = ld;
    A.M = 1;
    A.cap = cap;
    A.V = n_voxels;
    A.n_tot = (unsigned)n_rows;
    A.K = KB;
    DevCtx* ctx;
    if ((rc = current_ctx(&ctx)) != VPET_OK) return rc;
    hipStream_t st = (hipStream_t)hip_stream;
    std::lock_guard<std::mutex> lock(ctx->mu);
    int slot;
    const void* dom;
    if ((rc = upload_blob(*ctx, omega.data(), sizeof(double) * F, st, &dom, slot)) != VPET_OK) return rc;
    A.omega = static_cast<const double*>(dom);
    const size_t V = (size_t)n_voxels;
    const size_t sz_cnt = align256(sizeof(int) * 2 * V), sz_cand = align256(sizeof(uint64_t) * (size_t)cap * V);
    const size_t sz_b = align256(sizeof(uint16_t) * (size_t)KB * (size_t)n_rows);
    const size_t sz_a = align256(sizeof(uint16_t) * (size_t)KB * V);
    const size_t sz_c = align256(sizeof(float) * V), sz_av = align256(sizeof(double) * V);
    char* work = nullptr;
    hipError_t e = hipMallocAsync((void**)&work, sz_cnt + sz_cand + 2 * sz_b + 2 * sz_a + 4 * sz_c + sz_av, st);
    if (e != hipSuccess) return fail(VPET_E_NOMEM, "screen work: %s", hipGetErrorString(e));
    char* q = work;
    A.cnt = reinterpret_cast<int*>(q);
    A.cnt_hi = A.cnt + V;
    q += sz_cnt;
    A.cand = reinterpret_cast<uint64_t*>(q);
    q += sz_cand;
    A.bhi = reinterpret_cast<uint16_t*>(q);
    q += sz_b;
    A.blo = reinterpret_cast<uint16_t*>(q);
    q += sz_b;
    A.ahi = reinterpret_cast<uint16_t*>(q);
    q += sz_a;
    A.alo = reinterpret_cast<uint16_t*>(q);
    q += sz_a;
    A.cthr = reinterpret_cast<float*>(q);
    q += sz_c;
    A.cthr1 = reinterpret_cast<float*>(q);
    q += sz_c;
    A.tau = reinterpret_cast<float*>(q);
    q += sz_c;
    A.tau1 = reinterpret_cast<float*>(q);
    q += sz_c;
    A.aval = reinterpret_cast<double*>(q);
    const dim3 b256(256), rows((unsigned)((n_rows * (ld / 2) + 255) / 256)), lanes((unsigned)((V + 255) / 256));
    const dim3 mblocks((unsigned)((V + kMfmaVox - 1) / kMfmaVox)), per_voxel((unsigned)V);
#define VPET_SCREEN(LDV)                                                                   \
    do {                                                                                   \
        hipLaunchKernelGGL((vpet_bank_bops_kernel<LDV>), rows, b256, 0, st, A);            \
        hipLaunchKernelGGL((vpet_bank_aops_kernel<LDV>), lanes, b256, 0, st, A);           \
        hipLaunchKernelGGL(vpet_bank_passall_kernel, lanes, b256, 0, st, A);               \
        launch_mfma<2 * LDV, false>(mblocks, st, A);                                       \
    } while (0)
    switch (ld) {
        case 8: VPET_SCREEN(8); break;
        case 16: VPET_SCREEN(16); break;
        case 24: VPET_SCREEN(24); break;
        case 32: VPET_SCREEN(32); break;
        case 40: VPET_SCREEN(40); break;
        default: VPET_SCREEN(48); break;
    }
#undef VPET_SCREEN
    hipLaunchKernelGGL(vpet_bank_scatter_kernel, per_voxel, b256, 0, st, A, out_s, out_a);
    e = hipGetLastError();
    if (e != hipSuccess) rc = hip_fail(e, "screen launch");
    e = hipFreeAsync(work, st);
    if (e != hipSuccess && rc == VPET_OK) rc = hip_fail(e, "hipFreeAsync");
    e = hipEventRecord(ctx->ev[slot], st);
    if (e != hipSuccess && rc == VPET_OK) rc = hip_fail(e, "hipEventRecord");
    return rc;
}

// ===========================================================================
// Streaming driver: a volume in a file, two chunks in flight.
// ===========================================================================
}  // extern "C"

namespace {

bool pread_all(int fd, void* buf, size_t bytes, off_t off) {
    char* p = static_cast<char*>(buf);
    while (bytes > 0) {
        const ssize_t r = ::pread(fd, p, bytes, off);
        if (r <= 0) return false;
        p += r;
        bytes -= (size_t)r;
        off += r;
    }
    return true;
}

bool pwrite_all(int fd, const void* buf, size_t bytes, off_t off) {
    const char* p = static_cast<const char*>(buf);
    while (bytes > 0) {
        const ssize_t r = ::pwrite(fd, p, bytes, off);
        if (r <= 0) return false;
        p += r;
        bytes -= (size_t)r;
        off += r;
    }
    return true;
}

// The progress line names the run's kind and shape so that a resume cannot
// continue a different run.
std::string progress_line(const char* kind, int64_t V, int F, int M, int64_t chunk, int64_t done) {
    char buf[192];
    snprintf(buf, sizeof buf, "%s v1 voxels=%lld frames=%d models=%d chunk=%lld done=%lld\n", kind, (long long)V, F,
             M, (long long)chunk, (long long)done);
    return buf;
}

int write_progress(const std::string& path, const std::string& line) {
    const std::string tmp = path + ".tmp";
    const int fd = ::open(tmp.c_str(), O_WRONLY | O_CREAT | O_TRUNC, 0644);
    if (fd < 0) return fail(VPET_E_IO, "cannot write %s", tmp.c_str());
    const bool ok = pwrite_all(fd, line.data(), line.size(), 0) && ::fsync(fd) == 0;
    ::close(fd);
    if (!ok || ::rename(tmp.c_str(), path.c_str()) != 0) return fail(VPET_E_IO, "cannot update %s", path.c_str());
    return VPET_OK;
}

// Host and device buffers of the pipeline; released by the destructor.
struct StreamBuffers {
    float* h_in[2] = {nullptr, nullptr};
    float* h_mom[2] = {nullptr, nullptr};
    float* h_prob[2] = {nullptr, nullptr};
    float* d_in[2] = {nullptr, nullptr};
    float* d_mom[2] = {nullptr, nullptr};
    float* d_prob[2] = {nullptr, nullptr};
    hipEvent_t ev_in[2] = {nullptr, nullptr}, ev_done[2] = {nullptr, nullptr};
    hipStream_t copy = nullptr;
    int fds[3] = {-1, -1, -1};
    ~StreamBuffers() {
        if (copy) (void)hipStreamSynchronize(copy);
        for (int b = 0; b < 2; ++b) {
            if (ev_done[b]) (void)hipEventSynchronize(ev_done[b]);
            if (h_in[b]) (void)hipHostFree(h_in[b]);
            if (h_mom[b]) (void)hipHostFree(h_mom[b]);
            if (h_prob[b]) (void)hipHostFree(h_prob[b]);
            if (d_in[b]) (void)hipFree(d_in[b]);
            if (d_mom[b]) (void)hipFree(d_mom[b]);
            if (d_prob[b]) (void)hipFree(d_prob[b]);
            if (ev_in[b]) (void)hipEventDestroy(ev_in[b]);
            if (ev_done[b]) (void)hipEventDestroy(ev_done[b]);
        }
        if (copy) (void)hipStreamDestroy(copy);
        for (int fd : fds)
            if (fd >= 0) ::close(fd);
    }
};

}  // namespace

extern "C" {

}  // extern "C"

namespace {

// Runs `run` (device input chunk -> device output chunk, enqueued on st) over
// a volume in a file with two chunks in flight and resumable progress.
using ChunkRun = std::function<int(const float* d_in, int64_t rows, float* d_mom, float* d_prob, int64_t chunk)>;

int stream_driver(const char* kind, const char* tacs_path, int64_t n_voxels, int F, int M, int64_t chunk_voxels,
                  const char* out_prefix, int32_t resume, int64_t max_chunks, int64_t* out_done, hipStream_t st,
                  const ChunkRun& run) {
    int rc = VPET_OK;
    const int64_t chunk = std::min<int64_t>(chunk_voxels, std::max<int64_t>(n_voxels, 1));
    const int64_t nchunks = (n_voxels + chunk - 1) / chunk;
    const size_t in_row = sizeof(float) * (size_t)F, mom_row = sizeof(float) * (size_t)M * VPET_PSTRIDE * 2,
                 prob_row = sizeof(float) * (size_t)M;

    StreamBuffers B;
    B.fds[0] = ::open(tacs_path, O_RDONLY);
    if (B.fds[0] < 0) return fail(VPET_E_IO, "cannot open %s", tacs_path);
    struct stat st_in;
    if (::fstat(B.fds[0], &st_in) != 0 || (uint64_t)st_in.st_size < (uint64_t)n_voxels * in_row)
        return fail(VPET_E_IO, "%s holds fewer than %lld x %d fp32 values", tacs_path, (long long)n_voxels, F);
    const std::string pre(out_prefix), mom_path = pre + ".moments", prob_path = pre + ".prob",
                                         prog_path = pre + ".progress";
    int64_t done = 0;
    if (resume) {
        const int fd = ::open(prog_path.c_str(), O_RDONLY);
        if (fd >= 0) {
            char buf[256] = {0};
            const ssize_t r = ::pread(fd, buf, sizeof buf - 1, 0);
            ::close(fd);
            long long v = -1, c = -1, d = -1;
            int f = -1, m = -1;
            char kbuf[64] = {0};
            if (r <= 0 || sscanf(buf, "%63s v1 voxels=%lld frames=%d models=%d chunk=%lld done=%lld", kbuf, &v, &f, &m,
                                 &c, &d) != 6)
                return fail(VPET_E_IO, "unreadable progress file %s", prog_path.c_str());
            if (std::strcmp(kbuf, kind) != 0 || v != n_voxels || f != F || m != M || c != chunk || d < 0 ||
                d > nchunks)
                return fail(VPET_E_ARG, "progress file %s belongs to a run of another kind or shape", prog_path.c_str());
            done = d;
        }
    }
    const int oflags = O_RDWR | O_CREAT | (resume ? 0 : O_TRUNC);
    B.fds[1] = ::open(mom_path.c_str(), oflags, 0644);
    B.fds[2] = ::open(prob_path.c_str(), oflags, 0644);
    if (B.fds[1] < 0 || B.fds[2] < 0) return fail(VPET_E_IO, "cannot open %s.*", out_prefix);
    if (::ftruncate(B.fds[1], (off_t)(mom_row * (size_t)n_voxels)) != 0 ||
        ::ftruncate(B.fds[2], (off_t)(prob_row * (size_t)n_voxels)) != 0)
        return fail(VPET_E_IO, "cannot size the output files %s.*", out_prefix);
    if (!resume || done == 0)
        if ((rc = write_progress(prog_path, progress_line(kind, n_voxels, F, M, chunk, 0))) != VPET_OK) return rc;
    const int64_t last = max_chunks > 0 ? std::min<int64_t>(nchunks, done + max_chunks) : nchunks;
    if (done >= last) {
        if (out_done) *out_done = done;
        return VPET_OK;
    }

    hipError_t e = hipStreamCreateWithFlags(&B.copy, hipStreamNonBlocking);
    for (int b = 0; b < 2 && e == hipSuccess; ++b) {
        e = hipHostMalloc((void**)&B.h_in[b], in_row * chunk, hipHostMallocDefault);
        if (e == hipSuccess) e = hipHostMalloc((void**)&B.h_mom[b], mom_row * chunk, hipHostMallocDefault);
        if (e == hipSuccess) e = hipHostMalloc((void**)&B.h_prob[b], prob_row * chunk, hipHostMallocDefault);
        if (e == hipSuccess) e = hipMalloc((void**)&B.d_in[b], in_row * chunk);
        if (e == hipSuccess) e = hipMalloc((void**)&B.d_mom[b], mom_row * chunk);
        if (e == hipSuccess) e = hipMalloc((void**)&B.d_prob[b], prob_row * chunk);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&B.ev_in[b], hipEventDisableTiming);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&B.ev_done[b], hipEventDisableTiming);
    }
    if (e != hipSuccess) return fail(VPET_E_NOMEM, "stream buffers: %s", hipGetErrorString(e));

    auto rows = [&](int64_t c) { return std::min<int64_t>(chunk, n_voxels - c * chunk); };
    // read chunk c into host buffer b and queue its copy to the device
    auto load = [&](int64_t c, int b) -> int {
        hipError_t he = hipEventSynchronize(B.ev_in[b]);  // the previous copy out of h_in[b]
        if (he != hipSuccess) return hip_fail(he, "hipEventSynchronize");
        if (!pread_all(B.fds[0], B.h_in[b], in_row * (size_t)rows(c), (off_t)(in_row * (size_t)(c * chunk))))
            return fail(VPET_E_IO, "read of %s failed at chunk %lld", tacs_path, (long long)c);
        he = hipStreamWaitEvent(B.copy, B.ev_done[b], 0);  // d_in[b] free: its last chunk was screened
        if (he == hipSuccess)
            he = hipMemcpyAsync(B.d_in[b], B.h_in[b], in_row * (size_t)rows(c), hipMemcpyHostToDevice, B.copy);
        if (he == hipSuccess) he = hipEventRecord(B.ev_in[b], B.copy);
        return he == hipSuccess ? VPET_OK : hip_fail(he, "chunk copy in");
    };
    // wait for chunk c's outputs and write them at their offsets (writer thread)
    auto store = [&](int64_t c, int b) -> int {
        hipError_t he = hipEventSynchronize(B.ev_done[b]);
        if (he != hipSuccess) return hip_fail(he, "chunk outputs");
        const size_t n = (size_t)rows(c), v0 = (size_t)(c * chunk);
        if (!pwrite_all(B.fds[1], B.h_mom[b], mom_row * n, (off_t)(mom_row * v0)) ||
            !pwrite_all(B.fds[2], B.h_prob[b], prob_row * n, (off_t)(prob_row * v0)) || ::fsync(B.fds[1]) != 0 ||
            ::fsync(B.fds[2]) != 0)
            return fail(VPET_E_IO, "write of %s.* failed at chunk %lld", out_prefix, (long long)c);
        return write_progress(prog_path, progress_line(kind, n_voxels, F, M, chunk, c + 1));
    };

    // A writer thread writes, syncs and records the chunks' outputs in chunk
    // order, so that the file writes overlap both the GPU's work and the main
    // thread's reads.  Chunks [done, queued) are handed over, [done, written)
    // are on disk; its error (code and message) is passed back.
    struct Writer {
        std::mutex mu;
        std::condition_variable cv;
        int64_t queued = 0, written = 0;
        int rc = VPET_OK;
        std::string err;
        bool quit = false;
        std::thread th;
        ~Writer() {
            {
                std::lock_guard<std::mutex> lk(mu);
                quit = true;
            }
            cv.notify_all();
            if (th.joinable()) th.join();
        }
    } W;
    W.queued = W.written = done;
    try {
        W.th = std::thread([&] {
            for (;;) {
                int64_t c;
                {
                    std::unique_lock<std::mutex> lk(W.mu);
                    W.cv.wait(lk, [&] { return W.quit || W.written < W.queued; });
                    if (W.quit) return;
                    c = W.written;
                }
                const int r = store(c, (int)((c - done) & 1));
                {
                    std::lock_guard<std::mutex> lk(W.mu);
                    if (r != VPET_OK) {
                        W.rc = r;
                        W.err = g_err;
                        W.quit = true;
                    } else {
                        W.written = c + 1;
                    }
                }
                W.cv.notify_all();
                if (r != VPET_OK) return;
            }
        });
    } catch (...) {
        return fail(VPET_E_NOMEM, "cannot start the stream's writer thread");
    }
    // wait until the chunks below `upto` are on disk
    auto wait_written = [&](int64_t upto) -> int {
        std::unique_lock<std::mutex> lk(W.mu);
        W.cv.wait(lk, [&] { return W.written >= upto || W.rc != VPET_OK; });
        return W.rc == VPET_OK ? VPET_OK : fail(W.rc, "%s", W.err.c_str());
    };
    auto finish = [&](int r) {
        if (out_done) {
            std::lock_guard<std::mutex> lk(W.mu);
            *out_done = W.written;
        }
        return r;
    };

    if ((rc = load(done, 0)) != VPET_OK) return finish(rc);
    for (int64_t c = done; c < last; ++c) {
        const int b = (int)((c - done) & 1);
        e = hipStreamWaitEvent(st, B.ev_in[b], 0);
        if (e != hipSuccess) return finish(hip_fail(e, "hipStreamWaitEvent"));
        if ((rc = run(B.d_in[b], rows(c), B.d_mom[b], B.d_prob[b], c)) != VPET_OK) return finish(rc);
        // h_mom[b], h_prob[b] and ev_done[b] are chunk c - 2's until it is written
        if (c - 2 >= done && (rc = wait_written(c - 1)) != VPET_OK) return finish(rc);
        e = hipMemcpyAsync(B.h_mom[b], B.d_mom[b], mom_row * (size_t)rows(c), hipMemcpyDeviceToHost, st);
        if (e == hipSuccess)
            e = hipMemcpyAsync(B.h_prob[b], B.d_prob[b], prob_row * (size_t)rows(c), hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipEventRecord(B.ev_done[b], st);
        if (e != hipSuccess) return finish(hip_fail(e, "chunk copy out"));
        {
            std::lock_guard<std::mutex> lk(W.mu);
            W.queued = c + 1;
        }
        W.cv.notify_all();
        if (c + 1 < last && (rc = load(c + 1, b ^ 1)) != VPET_OK) return finish(rc);  // overlaps chunk c
    }
    return finish(wait_written(last));
}

}  // namespace

extern "C" {

int vpet_abc_stream_bank(const char* tacs_path, int64_t n_voxels, const float* frame_times, vpet_grid grid,
                         uint32_t model_id, int64_t n_draws, double accept_frac, const float* bank_theta,
                         const double* bank_x, int64_t chunk_voxels, const char* out_prefix, int32_t resume,
                         int64_t max_chunks, const vpet_abc_opts* opts, int64_t* out_done, void* hip_stream) {
    if (out_done) *out_done = 0;
    vpet_abc_opts o{};
    if (opts) o = *opts;
    if (o.weights || o.out_accept_idx || o.out_accept_dist || o.out_threshold || o.out_scan_ms ||
        o.out_fallback_voxels)
        return fail(VPET_E_ARG, "streaming takes no caller weights, debug outputs or reports");
    // everything vpet_abc_infer_bank checks, without work (0 voxels)
    int rc = vpet_abc_infer_bank(nullptr, 0, frame_times, grid, model_id, n_draws, accept_frac, bank_theta, bank_x,
                                 nullptr, nullptr, &o, hip_stream);
    if (rc != VPET_OK) return rc;
    if (!tacs_path || !out_prefix) return fail(VPET_E_ARG, "tacs_path and out_prefix must not be NULL");
    if (n_voxels < 0 || chunk_voxels < 1 || max_chunks < 0)
        return fail(VPET_E_ARG, "need n_voxels >= 0, chunk_voxels >= 1, max_chunks >= 0");
    if (!bank_theta || !bank_x) return fail(VPET_E_ARG, "bank pointers must not be NULL");
    const int F = grid.n_frames, M = __builtin_popcount(model_id);
    return stream_driver("vpet_abc_stream", tacs_path, n_voxels, F, M, chunk_voxels, out_prefix, resume, max_chunks,
                         out_done, (hipStream_t)hip_stream,
                         [&](const float* d_in, int64_t rows, float* d_mom, float* d_prob, int64_t) {
                             return vpet_abc_infer_bank(d_in, rows, frame_times, grid, model_id, n_draws, accept_frac,
                                                        bank_theta, bank_x, d_mom, d_prob, &o, hip_stream);
                         });
}

int vpet_abc_stream_bank_learned(const char* tacs_path, int64_t n_voxels, const float* frame_times,
                                 const float* input_fn, vpet_grid grid, uint32_t model_id, const double* prior_box,
                                 const float* params, const vpet_bank_groups* groups, int64_t n_draws,
                                 double accept_frac, uint64_t seed, int64_t chunk_voxels, const char* out_prefix,
                                 int32_t resume, int64_t max_chunks, const vpet_abc_opts* opts, int64_t* out_done,
                                 void* hip_stream) {
    if (out_done) *out_done = 0;
    vpet_abc_opts o{};
    if (opts) o = *opts;
    if (o.weights || o.out_accept_idx || o.out_accept_dist || o.out_threshold || o.out_scan_ms ||
        o.out_fallback_voxels || o.out_ess || o.accept_below)
        return fail(VPET_E_ARG, "streaming takes no caller weights, per-voxel inputs, debug outputs or reports");
    if (!groups) return fail(VPET_E_ARG, "groups must not be NULL");
    if (groups->out_group || groups->out_bank_theta || groups->out_bank_logw)
        return fail(VPET_E_ARG, "streaming takes no bank outputs");
    // everything vpet_abc_infer_bank_learned checks, without work (0 voxels)
    int rc = vpet_abc_infer_bank_learned(nullptr, 0, frame_times, input_fn, grid, model_id, prior_box, nullptr, groups,
                                         n_draws, accept_frac, seed, nullptr, nullptr, &o, hip_stream);
    if (rc != VPET_OK) return rc;
    if (!tacs_path || !out_prefix || !params)
        return fail(VPET_E_ARG, "tacs_path, out_prefix and params must not be NULL");
    if (grid.n_frames > 32) return fail(VPET_E_LIMIT, "the proposal network takes 1..32 frames");
    if (n_voxels < 0 || chunk_voxels < 1 || max_chunks < 0)
        return fail(VPET_E_ARG, "need n_voxels >= 0, chunk_voxels >= 1, max_chunks >= 0");
    const int F = grid.n_frames, M = __builtin_popcount(model_id);
    const int64_t chunk = std::min<int64_t>(chunk_voxels, std::max<int64_t>(n_voxels, 1));
    float* d_prop = nullptr;
    hipError_t e = hipMalloc((void**)&d_prop, sizeof(float) * VPET_PROPOSAL_NOUT * (size_t)chunk);
    if (e != hipSuccess) return fail(VPET_E_NOMEM, "proposal outputs: %s", hipGetErrorString(e));
    // chunk c's groups continue the numbering of the Philox counters
    const int64_t groups_per_chunk = (chunk + groups->group_voxels - 1) / groups->group_voxels;
    rc = stream_driver("vpet_abc_stream_learned", tacs_path, n_voxels, F, M, chunk_voxels, out_prefix, resume,
                       max_chunks, out_done, (hipStream_t)hip_stream,
                       [&](const float* d_in, int64_t rows, float* d_mom, float* d_prob, int64_t c) {
                           int r = vpet_proposal_forward(params, d_in, rows, F, d_prop, hip_stream);
                           if (r != VPET_OK) return r;
                           vpet_bank_groups gc = *groups;
                           gc.first_group = groups->first_group + c * groups_per_chunk;
                           return vpet_abc_infer_bank_learned(d_in, rows, frame_times, input_fn, grid, model_id,
                                                              prior_box, d_prop, &gc, n_draws, accept_frac, seed,
                                                              d_mom, d_prob, &o, hip_stream);
                       });
    // every chunk's work is done (the driver waited for the last outputs) or
    // the call failed; either way wait before freeing
    (void)hipStreamSynchronize((hipStream_t)hip_stream);
    (void)hipFree(d_prop);
    return rc;
}


// ===========================================================================
// Learned proposal: network evaluation and training.
// ===========================================================================
}  // extern "C"

namespace {

__global__ __launch_bounds__(256) void vpet_fill_kernel(float* p, long long n, float v) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

template <int D>
__global__ __launch_bounds__(256) void vpet_net_targets_kernel(const float* theta, long long n, float* Z) {
    const long long b = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= n) return;
    for (int j = 0; j < D; ++j) Z[b * D + j] = (float)log(fmax((double)theta[b * VPET_PSTRIDE + head_slot<D>(j)], 1e-6));
}

// Activations of one batch of up to `rows` samples.
struct NetWork {
    float *X, *H1, *H2, *O, *dO, *dH1, *dH2, *Z;
    float* part;  // split-K partials: kSplitMax tiles of at most kNetH x kNetH
    long long rows;
};

constexpr int kSplitMax = 16;

size_t net_work_bytes(long long rows) {
    return sizeof(float) * ((size_t)rows * (kNetIn + 4 * kNetH + 2 * kNetOut + kMixDMax) +
                            (size_t)kSplitMax * kNetH * kNetH) + 9 * 256;
}

void net_work_carve(char* base, long long rows, NetWork& w) {
    auto take = [&](size_t nfl) {
        float* p = reinterpret_cast<float*>(base);
        base += align256(sizeof(float) * nfl);
        return p;
    };
    w.rows = rows;
    w.X = take((size_t)rows * kNetIn);
    w.H1 = take((size_t)rows * kNetH);
    w.H2 = take((size_t)rows * kNetH);
    w.dH1 = take((size_t)rows * kNetH);
    w.dH2 = take((size_t)rows * kNetH);
    w.O = take((size_t)rows * kNetOut);
    w.dO = take((size_t)rows * kNetOut);
    w.Z = take((size_t)rows * kMixDMax);
    w.part = take((size_t)kSplitMax * kNetH * kNetH);
}

// A product with few output tiles and a long K (the weight gradients: K =
// batch rows) is split along K over up to kSplitMax blocks per tile, so that
// the launch fills the chip; the partials are added in a fixed order, which
// keeps the result deterministic.
void gemm(hipStream_t st, const float* A, long long sam, long long sak, const float* B, long long sbk, long long sbn,
          float* C, long long ldc, int M, int N, int K, const float* bias, int relu, const float* mask, long long ldm,
          float* part) {
    GemmArgs G{A, sam, sak, B, sbk, sbn, C, ldc, bias, mask, ldm, M, N, K, relu, 0, K, nullptr, 0};
    const int tiles = ((N + 63) / 64) * ((M + 63) / 64);
    int S = 1;
    if (part && tiles < 128 && K >= 512 && (long long)M * N <= (long long)kNetH * kNetH) {
        S = std::min(std::min(kSplitMax, (256 + tiles - 1) / tiles), K / 256);
        G.kchunk = ((K + S - 1) / S + 15) & ~15;
        S = (K + G.kchunk - 1) / G.kchunk;
    }
    if (S > 1) {
        G.part = part;
        G.pstride = (long long)M * N;
    }
    hipLaunchKernelGGL(vpet_gemm_bf16x3_kernel, dim3((unsigned)((N + 63) / 64), (unsigned)((M + 63) / 64), (unsigned)S),
                       dim3(256), 0, st, G);
    if (S > 1)
        hipLaunchKernelGGL(vpet_gemm_reduce_kernel, dim3((unsigned)(((long long)M * N + 255) / 256)), dim3(256), 0, st,
                           G, S);
}

// H1 = relu(X W1 + b1), H2 = relu(H1 W2 + b2), O = H2 W3 + b3 for n rows of X.
void net_forward(hipStream_t st, const float* p, const NetWork& w, int n) {
    gemm(st, w.X, kNetIn, 1, p + kOffW1, kNetH, 1, w.H1, kNetH, n, kNetH, kNetIn, p + kOffB1, 1, nullptr, 0, w.part);
    gemm(st, w.H1, kNetH, 1, p + kOffW2, kNetH, 1, w.H2, kNetH, n, kNetH, kNetH, p + kOffB2, 1, nullptr, 0, w.part);
    gemm(st, w.H2, kNetH, 1, p + kOffW3, kNetOut, 1, w.O, kNetOut, n, kNetOut, kNetH, p + kOffB3, 0, nullptr, 0, w.part);
}

// Gradients of the mean negative log density into g (overwritten), given dO.
void net_backward(hipStream_t st, const float* p, const NetWork& w, int n, float* g) {
    gemm(st, w.H2, 1, kNetH, w.dO, kNetOut, 1, g + kOffW3, kNetOut, kNetH, kNetOut, n, nullptr, 0, nullptr, 0, w.part);
    hipLaunchKernelGGL(vpet_colsum_kernel, dim3(kNetOut), dim3(256), 0, st, w.dO, (long long)kNetOut, n, g + kOffB3);
    gemm(st, w.dO, kNetOut, 1, p + kOffW3, 1, kNetOut, w.dH2, kNetH, n, kNetH, kNetOut, nullptr, 0, w.H2, kNetH, w.part);
    gemm(st, w.H1, 1, kNetH, w.dH2, kNetH, 1, g + kOffW2, kNetH, kNetH, kNetH, n, nullptr, 0, nullptr, 0, w.part);
    hipLaunchKernelGGL(vpet_colsum_kernel, dim3(kNetH), dim3(256), 0, st, w.dH2, (long long)kNetH, n, g + kOffB2);
    gemm(st, w.dH2, kNetH, 1, p + kOffW2, 1, kNetH, w.dH1, kNetH, n, kNetH, kNetH, nullptr, 0, w.H1, kNetH, w.part);
    gemm(st, w.X, 1, kNetIn, w.dH1, kNetH, 1, g + kOffW1, kNetH, kNetIn, kNetH, n, nullptr, 0, nullptr, 0, w.part);
    hipLaunchKernelGGL(vpet_colsum_kernel, dim3(kNetH), dim3(256), 0, st, w.dH1, (long long)kNetH, n, g + kOffB1);
}

int check_frames(int32_t n_frames) {
    if (n_frames < 1 || n_frames > kNetIn) return fail(VPET_E_LIMIT, "the proposal network takes 1..%d frames", kNetIn);
    return VPET_OK;
}

unsigned long long gcd_u64(unsigned long long a, unsigned long long b) {
    while (b) {
        const unsigned long long t = a % b;
        a = b;
        b = t;
    }
    return a;
}

}  // namespace

extern "C" {

int vpet_proposal_init(float* params, uint64_t seed, void* hip_stream) {
    if (!params) return fail(VPET_E_ARG, "params must not be NULL");
    hipLaunchKernelGGL(vpet_net_init_kernel, dim3((unsigned)((kNetParams + 255) / 256)), dim3(256), 0,
                       (hipStream_t)hip_stream, params, (uint32_t)seed, (uint32_t)(seed >> 32));
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? VPET_OK : hip_fail(e, "proposal init");
}

int vpet_proposal_forward(const float* params, const float* tacs, int64_t n, int32_t n_frames, float* out,
                          void* hip_stream) {
    int rc = check_frames(n_frames);
    if (rc != VPET_OK) return rc;
    if (n < 0) return fail(VPET_E_ARG, "n must be >= 0");
    if (n == 0) return VPET_OK;
    if (!params || !tacs || !out) return fail(VPET_E_ARG, "params, tacs and out must not be NULL");
    int dev;
    if ((rc = current_device(&dev)) != VPET_OK) return rc;
    hipStream_t st = (hipStream_t)hip_stream;
    const long long rows = std::min<long long>(n, 1LL << 17);
    char* work = nullptr;
    hipError_t e = hipMallocAsync((void**)&work, net_work_bytes(rows), st);
    if (e != hipSuccess) return fail(VPET_E_NOMEM, "proposal work: %s", hipGetErrorString(e));
    NetWork w;
    net_work_carve(work, rows, w);
    for (long long b0 = 0; b0 < n; b0 += rows) {
        const int cnt = (int)std::min<long long>(rows, n - b0);
        hipLaunchKernelGGL(vpet_net_features_kernel, dim3((unsigned)((cnt + 255) / 256)), dim3(256), 0, st,
                           tacs + (size_t)b0 * n_frames, (long long)cnt, n_frames, w.X);
        NetWork wo = w;
        wo.O = out + (size_t)b0 * kNetOut;  // the last layer writes the caller's buffer
        net_forward(st, params, wo, cnt);
    }
    e = hipGetLastError();
    const hipError_t e2 = hipFreeAsync(work, st);
    if (e != hipSuccess) return hip_fail(e, "proposal forward");
    return e2 == hipSuccess ? VPET_OK : hip_fail(e2, "hipFreeAsync");
}

int vpet_proposal_loss_grad(const float* params, const float* tacs, const float* theta, int64_t n, int32_t n_frames,
                            int32_t dims, float* grad, float* loss, void* hip_stream) {
    int rc = check_frames(n_frames);
    if (rc != VPET_OK) return rc;
    if (dims != 4 && dims != 5) return fail(VPET_E_ARG, "dims must be 4 or 5");
    if (n < 1 || n > (1LL << 20)) return fail(VPET_E_ARG, "n must lie in [1, 2^20]");
    if (!params || !tacs || !theta || !grad || !loss) return fail(VPET_E_ARG, "pointers must not be NULL");
    int dev;
    if ((rc = current_device(&dev)) != VPET_OK) return rc;
    hipStream_t st = (hipStream_t)hip_stream;
    char* work = nullptr;
    hipError_t e = hipMallocAsync((void**)&work, net_work_bytes(n), st);
    if (e != hipSuccess) return fail(VPET_E_NOMEM, "proposal work: %s", hipGetErrorString(e));
    NetWork w;
    net_work_carve(work, n, w);
    const unsigned blk = (unsigned)((n + 255) / 256);
    hipLaunchKernelGGL(vpet_net_features_kernel, dim3(blk), dim3(256), 0, st, tacs, (long long)n, n_frames, w.X);
    if (dims == 4)
        hipLaunchKernelGGL(vpet_net_targets_kernel<4>, dim3(blk), dim3(256), 0, st, theta, (long long)n, w.Z);
    else
        hipLaunchKernelGGL(vpet_net_targets_kernel<5>, dim3(blk), dim3(256), 0, st, theta, (long long)n, w.Z);
    hipLaunchKernelGGL(vpet_fill_kernel, dim3(1), dim3(256), 0, st, loss, 1LL, 0.0f);
    net_forward(st, params, w, (int)n);
    if (dims == 4)
        hipLaunchKernelGGL(vpet_mix_loss_kernel<4>, dim3(blk), dim3(256), 0, st, w.O, w.Z, (int)n, w.dO, loss);
    else
        hipLaunchKernelGGL(vpet_mix_loss_kernel<5>, dim3(blk), dim3(256), 0, st, w.O, w.Z, (int)n, w.dO, loss);
    net_backward(st, params, w, (int)n, grad);
    e = hipGetLastError();
    const hipError_t e2 = hipFreeAsync(work, st);
    if (e != hipSuccess) return hip_fail(e, "proposal loss/gradient");
    return e2 == hipSuccess ? VPET_OK : hip_fail(e2, "hipFreeAsync");
}

int vpet_proposal_train(float* params, const float* bank_theta, const double* bank_x, int64_t n_bank,
                        const float* frame_times, int32_t n_frames, int32_t dims, double noise_level,
                        double decay_lambda, int64_t steps, int32_t batch, float learning_rate, uint64_t seed,
                        float* out_loss, void* hip_stream) {
    const int F = n_frames;
    int rc = check_frames(F);
    if (rc != VPET_OK) return rc;
    if (dims != 4 && dims != 5) return fail(VPET_E_ARG, "dims must be 4 or 5");
    if (!params || !bank_theta || !bank_x || !frame_times) return fail(VPET_E_ARG, "pointers must not be NULL");
    if (n_bank < 1 || n_bank > 4294967295LL || steps < 0 || batch < 1 || batch > (1 << 20))
        return fail(VPET_E_ARG, "need 1 <= n_bank < 2^32, steps >= 0, 1 <= batch <= 2^20");
    if (!(learning_rate > 0.0f) || !(noise_level >= 0.0) || !(decay_lambda >= 0.0))
        return fail(VPET_E_ARG, "learning_rate > 0, noise_level >= 0 and decay_lambda >= 0 are required");
    std::vector<double> fac(kNetIn, 0.0);
    for (int f = 0; f < F; ++f) {
        const double a = frame_times[f], b = frame_times[f + 1];
        if (!(std::isfinite(a) && std::isfinite(b) && b > a)) return fail(VPET_E_GRID, "frame bounds must increase");
        fac[f] = noise_level * std::exp(decay_lambda * 0.5 * (a + b)) / (b - a);
    }
    if (steps == 0) return VPET_OK;
    const int ld = vpet_abc_bank_ld(F);
    DevCtx* ctx;
    if ((rc = current_ctx(&ctx)) != VPET_OK) return rc;
    hipStream_t st = (hipStream_t)hip_stream;
    std::lock_guard<std::mutex> lock(ctx->mu);
    int slot;
    const void* dfac;
    if ((rc = upload_blob(*ctx, fac.data(), sizeof(double) * kNetIn, st, &dfac, slot)) != VPET_OK) return rc;
    const size_t pbytes = align256(sizeof(float) * kNetParams);
    char* work = nullptr;
    hipError_t e = hipMallocAsync((void**)&work, 3 * pbytes + align256(sizeof(float) * (size_t)steps) +
                                                        net_work_bytes(batch), st);
    if (e != hipSuccess) return fail(VPET_E_NOMEM, "training work: %s", hipGetErrorString(e));
    float* g = reinterpret_cast<float*>(work);
    float* m = reinterpret_cast<float*>(work + pbytes);
    float* v = reinterpret_cast<float*>(work + 2 * pbytes);
    float* losses = reinterpret_cast<float*>(work + 3 * pbytes);
    NetWork w;
    net_work_carve(work + 3 * pbytes + align256(sizeof(float) * (size_t)steps), batch, w);
    const unsigned pblk = (unsigned)((kNetParams + 255) / 256);
    hipLaunchKernelGGL(vpet_fill_kernel, dim3(pblk), dim3(256), 0, st, m, (long long)kNetParams, 0.0f);
    hipLaunchKernelGGL(vpet_fill_kernel, dim3(pblk), dim3(256), 0, st, v, (long long)kNetParams, 0.0f);
    hipLaunchKernelGGL(vpet_fill_kernel, dim3((unsigned)((steps + 255) / 256)), dim3(256), 0, st, losses,
                       (long long)steps, 0.0f);
    const unsigned long long N = (unsigned long long)n_bank;
    unsigned long long mul = 1, add = 0;
    long long epoch = -1;
    const uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
    double b1t = 1.0, b2t = 1.0;
    for (long long t = 0; t < steps; ++t) {
        const unsigned long long j = (unsigned long long)t * (unsigned long long)batch;
        if ((long long)(j / N) != epoch) {  // a new pass over the bank: a new affine permutation of its rows
            epoch = (long long)(j / N);
            uint32_t hw[4];
            uint32_t c0 = (uint32_t)epoch, key0 = k0, key1 = k1, c1 = 0u, c2 = 6u, c3 = 0u;
            for (int r = 0; r < 10; ++r) {  // the same Philox4x32-10 on the host
                const uint64_t p0 = (uint64_t)0xD2511F53u * c0, p1 = (uint64_t)0xCD9E8D57u * c2;
                const uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ key0, n2 = (uint32_t)(p0 >> 32) ^ c3 ^ key1;
                c1 = (uint32_t)p1;
                c3 = (uint32_t)p0;
                c0 = n0;
                c2 = n2;
                key0 += 0x9E3779B9u;
                key1 += 0xBB67AE85u;
            }
            hw[0] = c0;
            hw[1] = c1;
            mul = N > 1 ? (((unsigned long long)hw[0] << 32 | hw[1]) % (N - 1)) + 1 : 1;
            while (gcd_u64(mul, N) != 1) mul = mul % N + 1;
            add = N > 1 ? (unsigned long long)c2 % N : 0;
        }
        const unsigned blk = (unsigned)((batch + 255) / 256);
        if (dims == 4)
            hipLaunchKernelGGL(vpet_net_batch_kernel<4>, dim3(blk), dim3(256), 0, st, bank_theta, bank_x, ld,
                               (long long)n_bank, F, static_cast<const double*>(dfac), j % N, mul, add, (uint32_t)epoch,
                               (int)batch, k0, k1, w.X, w.Z);
        else
            hipLaunchKernelGGL(vpet_net_batch_kernel<5>, dim3(blk), dim3(256), 0, st, bank_theta, bank_x, ld,
                               (long long)n_bank, F, static_cast<const double*>(dfac), j % N, mul, add, (uint32_t)epoch,
                               (int)batch, k0, k1, w.X, w.Z);
        net_forward(st, params, w, batch);
        if (dims == 4)
            hipLaunchKernelGGL(vpet_mix_loss_kernel<4>, dim3(blk), dim3(256), 0, st, w.O, w.Z, (int)batch, w.dO,
                               losses + t);
        else
            hipLaunchKernelGGL(vpet_mix_loss_kernel<5>, dim3(blk), dim3(256), 0, st, w.O, w.Z, (int)batch, w.dO,
                               losses + t);
        net_backward(st, params, w, batch, g);
        b1t *= 0.9;
        b2t *= 0.999;
        const double lr_t = learning_rate * 0.5 * (1.0 + std::cos(M_PI * (double)t / (double)steps));
        hipLaunchKernelGGL(vpet_adam_kernel, dim3(pblk), dim3(256), 0, st, params, g, m, v, (long long)kNetParams,
                           (float)lr_t, (float)(1.0 / (1.0 - b1t)), (float)(1.0 / (1.0 - b2t)));
        e = hipGetLastError();
        if (e != hipSuccess) break;
    }
    if (e == hipSuccess && out_loss)
        e = hipMemcpyAsync(out_loss, losses, sizeof(float) * (size_t)steps, hipMemcpyDeviceToHost, st);
    const hipError_t e2 = hipFreeAsync(work, st);
    const hipError_t e3 = hipEventRecord(ctx->ev[slot], st);
    if (e == hipSuccess && out_loss) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return hip_fail(e, "proposal training");
    if (e2 != hipSuccess) return hip_fail(e2, "hipFreeAsync");
    return e3 == hipSuccess ? VPET_OK : hip_fail(e3, "hipEventRecord");
}

}  // extern "C"
