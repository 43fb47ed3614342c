#pragma once
// Device code shared by the loop-hafnian kernels (gfx950 / CDNA4): complex
// arithmetic, wavefront cross-lane sums and the per-subset kernel template.
//
// Method (Quesada et al., arXiv:2010.15595, Sec. IV; algorithm of its
// Ref. [bjorklund2018faster]): with N = 2n, pairs (i, i+n), A0 = A with zero
// diagonal and d = diag(A), for every pair subset S of size s (m = 2s)
//     C = X_S A0_S,   c_k = tr(C^k) / (2k) + d_S^T C^(k-1) X_S d_S / 2,
//     t_S = (-1)^(n-s) [eta^n] exp(sum_k c_k eta^k),       lhaf = sum_S t_S.
//
// GPU formulation (differs from the paper's CPU code, same value):
//  * The loop terms come from a bordered determinant instead of mat-vecs:
//    with C' = [[0, d_S^T], [X_S d_S, C]],
//        det(I - eta C') = det(I - eta C) (1 - eta^2 d^T (I - eta C)^-1 X d),
//    so sum_k q_k eta^k = (R(eta) - R'(eta)) / (eta R(eta)) with
//    R = det(I - eta C), R' = det(I - eta C').
//  * C' is reduced to upper Hessenberg H' by Householder reflectors in
//    registers: the border column is the first reflector (it maps X d to a
//    multiple of e_1), then the Householder steps of C; the border row only
//    receives right applications.  H'[1:,1:] is similar to C, H' to C'.
//  * La Budde's recurrence (Rehman & Ipsen 2011) is run over the trailing
//    principal blocks of H' (expansion along the first row of each trailing
//    block), so one pass yields both det(xI - C) and det(xI - C').  Only the
//    n+2 leading coefficients are carried (lane d holds the coefficient of
//    x^(size-d)).
//  * A second kernel (one lane per subset) forms the power traces by Newton's
//    identities, the loop terms by power-series division, and the
//    exp-series coefficient; partial sums are compensated (TwoSum) and reduced
//    in a fixed order, so results are bitwise reproducible.
//
// Register layout of the m x m Hessenberg work: a wavefront holds W = 64/(P Q)
// subsets of one size class; lane l = g (P Q) + pc P + pr serves subset g and
// owns rows r = pr + P i (i < MR) and columns c = pc + Q k (k < MC).  Column
// sums reduce over the P consecutive lanes (DPP quad_perm / row_half_mirror),
// row sums over the Q lanes of stride P (DPP row_ror plus the gfx950
// permlane16/32 swaps); a few 8x4 instances use the column-swap map instead
// (LaneMap below).  Lane grids: 8x8 (one subset per wave), 8x4 (two), 4x4
// (four); the choice per subset size is made by the host (autotuned).

#include "lhaf_kernels.h"

namespace gbs {

// ---------------------------------------------------------------- complex

__device__ __forceinline__ double2 cz() { return make_double2(0.0, 0.0); }
__device__ __forceinline__ double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ double2 cscale(double2 a, double s) { return make_double2(a.x * s, a.y * s); }
__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
    return make_double2(fma(a.x, b.x, -a.y * b.y), fma(a.x, b.y, a.y * b.x));
}
// c + a * b
__device__ __forceinline__ double2 cfma(double2 a, double2 b, double2 c) {
    return make_double2(fma(a.x, b.x, fma(-a.y, b.y, c.x)), fma(a.x, b.y, fma(a.y, b.x, c.y)));
}
// c - a * b
__device__ __forceinline__ double2 cfms(double2 a, double2 b, double2 c) {
    return make_double2(fma(-a.x, b.x, fma(a.y, b.y, c.x)), fma(-a.x, b.y, fma(-a.y, b.x, c.y)));
}
// c + conj(a) * b
__device__ __forceinline__ double2 cfma_ca(double2 a, double2 b, double2 c) {
    return make_double2(fma(a.x, b.x, fma(a.y, b.y, c.x)), fma(a.x, b.y, fma(-a.y, b.x, c.y)));
}
// c - a * conj(b)
__device__ __forceinline__ double2 cfms_cb(double2 a, double2 b, double2 c) {
    return make_double2(fma(-a.x, b.x, fma(-a.y, b.y, c.x)), fma(a.x, b.y, fma(-a.y, b.x, c.y)));
}
__device__ __forceinline__ double cabs2(double2 a) { return fma(a.x, a.x, a.y * a.y); }

// ---------------------------------------------------------------- cross-lane

template <int CTRL>
__device__ __forceinline__ double dpp_mov(double x) {
    int lo = __builtin_amdgcn_mov_dpp(__double2loint(x), CTRL, 0xF, 0xF, false);
    int hi = __builtin_amdgcn_mov_dpp(__double2hiint(x), CTRL, 0xF, 0xF, false);
    return __hiloint2double(hi, lo);
}
template <int CTRL>
__device__ __forceinline__ float dpp_mov(float x) {
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(x), CTRL, 0xF, 0xF, false));
}

// Sum over the 8 lanes of an aligned octet; every lane of the octet gets the
// same bits (each butterfly level adds the same two operands, commuted).
__device__ __forceinline__ double sum_octet(double x) {
    x += dpp_mov<0x141>(x);  // row_half_mirror: lane i <- lane 7 - i
    x += dpp_mov<0xB1>(x);   // quad_perm [1,0,3,2]
    x += dpp_mov<0x4E>(x);   // quad_perm [2,3,0,1]
    return x;
}

__device__ __forceinline__ double swap_sum16(double x) {
    unsigned lo = (unsigned)__double2loint(x), hi = (unsigned)__double2hiint(x);
    auto l = __builtin_amdgcn_permlane16_swap(lo, lo, false, false);
    auto h = __builtin_amdgcn_permlane16_swap(hi, hi, false, false);
    return __hiloint2double((int)h[0], (int)l[0]) + __hiloint2double((int)h[1], (int)l[1]);
}

__device__ __forceinline__ double swap_sum32(double x) {
    unsigned lo = (unsigned)__double2loint(x), hi = (unsigned)__double2hiint(x);
    auto l = __builtin_amdgcn_permlane32_swap(lo, lo, false, false);
    auto h = __builtin_amdgcn_permlane32_swap(hi, hi, false, false);
    return __hiloint2double((int)h[0], (int)l[0]) + __hiloint2double((int)h[1], (int)l[1]);
}

// Register swaps across rows (16 lanes) and halves (32 lanes), gfx950:
//   swap16(x, y): x <- [x.r0, y.r0, x.r2, y.r2], y <- [x.r1, y.r1, x.r3, y.r3]
//   swap32(x, y): x <- [x.lo, y.lo],             y <- [x.hi, y.hi]
// (rK = lanes 16K..16K+15, lo/hi = lanes 0..31 / 32..63; checked by gbs_selftest).
__device__ __forceinline__ void swap16(double& x, double& y) {
    auto l = __builtin_amdgcn_permlane16_swap((unsigned)__double2loint(x), (unsigned)__double2loint(y), false, false);
    auto h = __builtin_amdgcn_permlane16_swap((unsigned)__double2hiint(x), (unsigned)__double2hiint(y), false, false);
    x = __hiloint2double((int)h[0], (int)l[0]);
    y = __hiloint2double((int)h[1], (int)l[1]);
}
__device__ __forceinline__ void swap32(double& x, double& y) {
    auto l = __builtin_amdgcn_permlane32_swap((unsigned)__double2loint(x), (unsigned)__double2loint(y), false, false);
    auto h = __builtin_amdgcn_permlane32_swap((unsigned)__double2hiint(x), (unsigned)__double2hiint(y), false, false);
    x = __hiloint2double((int)h[0], (int)l[0]);
    y = __hiloint2double((int)h[1], (int)l[1]);
}

// Sum over the 8 lanes {l mod 8 + 8 q : q = 0..7}.
__device__ __forceinline__ double sum_stride8(double x) {
    x += dpp_mov<0x128>(x);  // row_ror:8 -> partner lane l ^ 8
    x = swap_sum16(x);       // partner l ^ 16
    x = swap_sum32(x);       // partner l ^ 32
    return x;
}

__device__ __forceinline__ double2 csum_octet(double2 a) { return make_double2(sum_octet(a.x), sum_octet(a.y)); }
__device__ __forceinline__ double2 csum_stride8(double2 a) { return make_double2(sum_stride8(a.x), sum_stride8(a.y)); }

__device__ __forceinline__ double readlane_d(double x, int lane) {
    int lo = __builtin_amdgcn_readlane(__double2loint(x), lane);
    int hi = __builtin_amdgcn_readlane(__double2hiint(x), lane);
    return __hiloint2double(hi, lo);
}
__device__ __forceinline__ double2 readlane_c(double2 a, int lane) {
    return make_double2(readlane_d(a.x, lane), readlane_d(a.y, lane));
}

// Order LDS traffic between the lanes of one wavefront (no block barrier).
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ int uniform(int x) { return __builtin_amdgcn_readfirstlane(x); }

// ---------------------------------------------------------------- subsets

// s-subset of {0..n-1} with colexicographic rank `rank`:
// rank = sum_i C(c_i, i) over its elements c_1 < ... < c_s.
__device__ __forceinline__ uint64_t unrank_colex(uint64_t rank, int n, int s, const uint64_t* __restrict__ binom) {
    uint64_t mask = 0;
    int c = n - 1;
    for (int i = s; i >= 1; --i) {
        while (binom[c * kBinomStride + i] > rank) --c;
        mask |= 1ull << c;
        rank -= binom[c * kBinomStride + i];
        --c;
    }
    return mask;
}

// The s-subset following `mask` in colexicographic order (the next larger
// integer with the same number of set bits; Gosper's successor).  mask != 0.
__device__ __forceinline__ uint64_t colex_next(uint64_t mask) {
    const uint64_t ripple = mask + (mask & (~mask + 1ull));
    return ripple | (((ripple ^ mask) >> 2) >> __builtin_ctzll(mask));
}

// ---------------------------------------------------------------- phase 1

// Lane grids.  A wavefront holds W = 64 / (P Q) subsets of one size class.  Lane
// l serves subset group g and owns rows r = pr + P i (i < MR) and columns
// c = pc + Q k (k < MC) of its subset's matrix; column sums run over the P lanes
// of one (g, pc), row sums over the Q lanes of one (g, pr).
//  * Default map: l = g P Q + pc P + pr.  Column sums over P consecutive lanes
//    (DPP), row sums over stride P (DPP row_ror, permlane swaps).
//  * Column-swap map (CS, 8 x 4 grid): l = 8 pr + 4 g + pc.  Column sums run
//    over lane bits 3..5 (row_ror:8 and the two permlane swaps, which reduce
//    two columns for about the price of one), row sums over lane bits 0..1 (DPP
//    quad permutations).  It issues fewer instructions and holds fewer
//    registers; it is used where that gains an instance a wave per SIMD (the
//    8 x 4 tiles of 7 and 8 local columns with C at offset 0, with either La
//    Budde team width, and the one-team 3 x 6 tile at offset 0 together with
//    charpoly_min_waves), since elsewhere its longer chains of dependent swaps
//    cost more than the instructions it saves.
template <int P, int Q, bool CS>
struct LaneMap {
    __device__ static int pr(int l) { return l % P; }
    __device__ static int pc(int l) { return (l / P) % Q; }
    __device__ static int g(int l) { return l / (P * Q); }
};
template <>
struct LaneMap<8, 4, true> {
    __device__ static int pr(int l) { return l >> 3; }
    __device__ static int pc(int l) { return l & 3; }
    __device__ static int g(int l) { return (l >> 2) & 1; }
};
template <int P, int Q, int MR, int MC, int TEAM, int O>
constexpr bool lane_map_cs() {
    return P == 8 && Q == 4 && O == 0 && ((MR == 4 && MC >= 7) || (MR == 3 && MC == 6 && TEAM == 64));
}
// Waves per SIMD the compiler is held to: the FP64 one-team 8 x 4 instance with
// the 3 x 6 tile at offset 0 takes 172 registers with the column-swap map, 4
// above the three-wave limit; held to three waves it spills two of them (8
// bytes of scratch per lane) and runs 12% faster than at two waves.
template <int P, int Q, int MR, int MC, class V, int TEAM, int O>
constexpr int charpoly_min_waves() {
    return (P == 8 && Q == 4 && MR == 3 && MC == 6 && TEAM == 64 && O == 0 && sizeof(V) == sizeof(double2)) ? 3 : 1;
}

// Sums of NV values over the 8 lanes {l mod 8 + 8 q : q = 0..7}, all at once.
// The swap levels (lane ^ 32, then lane ^ 16) move values in pairs: each leaves
// every lane with half of the values summed over its partner (reduce-scatter);
// the lane ^ 8 level is a DPP butterfly; the same swaps run backwards to hand
// every lane all NV totals (all-gather).  Each total is formed in one place
// and copied, so all 8 lanes end with the same bits.
template <int NV>
__device__ __forceinline__ void stride8_sum_many(double (&v)[NV]) {
    static_assert(NV % 2 == 0, "even number of values");
    constexpr int NA = NV / 2, NB = (NA + 1) / 2;
    double a[NA], b[NB];
#pragma unroll
    for (int j = 0; j < NA; ++j) {
        double x = v[2 * j], y = v[2 * j + 1];
        swap32(x, y);
        a[j] = x + y;  // lanes 0..31: total of v[2j]; lanes 32..63: of v[2j+1]
    }
#pragma unroll
    for (int j = 0; j < NB; ++j) {
        double x = a[2 * j], y = (2 * j + 1 < NA) ? a[2 * j + 1] : 0.0;
        swap16(x, y);
        b[j] = x + y;  // even rows: a[2j], odd rows: a[2j+1]
    }
#pragma unroll
    for (int j = 0; j < NB; ++j) b[j] += dpp_mov<0x128>(b[j]);  // row_ror:8 (lane ^ 8)
#pragma unroll
    for (int j = 0; j < NB; ++j) {
        double x = b[j], y = b[j];
        swap16(x, y);
        a[2 * j] = x;
        if (2 * j + 1 < NA) a[2 * j + 1] = y;
    }
#pragma unroll
    for (int j = 0; j < NA; ++j) {
        double x = a[j], y = a[j];
        swap32(x, y);
        v[2 * j] = x;
        v[2 * j + 1] = y;
    }
}

// Sum over the P lanes of one column group.  Each level adds two values that
// the partner lane adds in the other order, so all P lanes end with the same
// bits.
template <int P, bool CS>
__device__ __forceinline__ double sum_cols(double x) {
    if constexpr (CS) {
        return sum_stride8(x);
    } else {
        if constexpr (P == 8) x += dpp_mov<0x141>(x);  // row_half_mirror
        x += dpp_mov<0xB1>(x);                          // quad_perm [1,0,3,2]
        x += dpp_mov<0x4E>(x);                          // quad_perm [2,3,0,1]
        return x;
    }
}

// Column sums of NV values at once.
template <int P, bool CS, int NV>
__device__ __forceinline__ void colsum_many(double (&v)[NV]) {
    if constexpr (CS) {
        stride8_sum_many<NV>(v);
    } else {
#pragma unroll
        for (int j = 0; j < NV; ++j) v[j] = sum_cols<P, false>(v[j]);
    }
}

// Sum over the Q lanes of one row group (same bits in all Q lanes).
template <int P, int Q, bool CS>
__device__ __forceinline__ double sum_rows(double x) {
    if constexpr (CS) {
        x += dpp_mov<0xB1>(x);   // quad_perm [1,0,3,2] (lane ^ 1)
        x += dpp_mov<0x4E>(x);   // quad_perm [2,3,0,1] (lane ^ 2)
    } else if constexpr (P == 8 && Q == 8) {
        x += dpp_mov<0x128>(x);  // row_ror:8 (lane ^ 8)
        x = swap_sum16(x);       // lane ^ 16
        x = swap_sum32(x);       // lane ^ 32
    } else if constexpr (P == 8 && Q == 4) {
        x += dpp_mov<0x128>(x);
        x = swap_sum16(x);
    } else if constexpr (P == 4 && Q == 4) {
        x += dpp_mov<0x128>(x);  // pair sums, equal in lanes i and i ^ 8
        x += dpp_mov<0x124>(x);  // row_ror:4 adds the other pair
    } else {
        static_assert(P == 4 && Q == 8, "unsupported lane grid");
        x += dpp_mov<0x128>(x);
        x += dpp_mov<0x124>(x);
        x = swap_sum16(x);
    }
    return x;
}

// Row sums of NV values at once.  Where a level crosses rows or halves
// (permlane swaps), values travel in pairs: each swap level leaves every lane
// with half of the values summed over its partner (reduce-scatter), the
// in-row level is a DPP butterfly, and the same swaps run backwards to hand
// every lane all NV totals (all-gather).  Each total is formed in one place
// and copied, so all Q lanes end with the same bits.
template <int P, int Q, bool CS, int NV>
__device__ __forceinline__ void rowsum_many(double (&v)[NV]) {
    static_assert(NV % 2 == 0, "even number of values");
    if constexpr (!CS && P == 8 && Q == 8) {
        stride8_sum_many<NV>(v);
    } else if constexpr (!CS && P == 8 && Q == 4) {
        constexpr int NB = NV / 2;
        double b[NB];
#pragma unroll
        for (int j = 0; j < NB; ++j) {
            double x = v[2 * j], y = v[2 * j + 1];
            swap16(x, y);
            b[j] = x + y;
        }
#pragma unroll
        for (int j = 0; j < NB; ++j) b[j] += dpp_mov<0x128>(b[j]);
#pragma unroll
        for (int j = 0; j < NB; ++j) {
            double x = b[j], y = b[j];
            swap16(x, y);
            v[2 * j] = x;
            v[2 * j + 1] = y;
        }
    } else {
#pragma unroll
        for (int j = 0; j < NV; ++j) v[j] = sum_rows<P, Q, CS>(v[j]);
    }
}

// Left application of a reflector to local columns K .. MC-1 over local rows
// I0 .. MR-1: w_k = sum_i conj(v_i) a[i][k] (a column sum), a[i][k] -= v_i w_k.
// With the column-swap map two columns are reduced together.
template <int P, bool CS, int MR, int MC, int I0, int K>
__device__ __forceinline__ void left_apply(double2 (&a)[MR][MC], const double2 (&vr)[MR]) {
    if constexpr (K < MC) {
        constexpr int NK = (CS && K + 1 < MC) ? 2 : 1;
        double v[2 * NK];
#pragma unroll
        for (int q = 0; q < NK; ++q) {
            double2 w = cz();
#pragma unroll
            for (int i = I0; i < MR; ++i) w = cfma_ca(vr[i], a[i][K + q], w);
            v[2 * q] = w.x;
            v[2 * q + 1] = w.y;
        }
        colsum_many<P, CS, 2 * NK>(v);
#pragma unroll
        for (int q = 0; q < NK; ++q) {
            const double2 w = make_double2(v[2 * q], v[2 * q + 1]);
#pragma unroll
            for (int i = I0; i < MR; ++i) a[i][K + q] = cfms(vr[i], w, a[i][K + q]);
        }
        left_apply<P, CS, MR, MC, I0, K + NK>(a, vr);
    }
}

// Right application of a reflector: u_i = sum_k a[i][k] vc[k] for every local
// row, and (WY) the border-row product sum_k y[k] vc[k], reduced together.
// Without WY the border row is a row of the tile (tiles with spare rows in
// front keep it in the row just above C) and needs nothing extra.
template <int P, int Q, bool CS, int MR, int MC, int K0, bool WY = true>
__device__ __forceinline__ void right_apply(double2 (&a)[MR][MC], double2 (&y)[MC], const double2 (&vc)[MC]) {
    constexpr int NV = 2 * MR + (WY ? 2 : 0);
    double v[NV];
#pragma unroll
    for (int i = 0; i < MR; ++i) {
        double2 u = cz();
#pragma unroll
        for (int k = K0; k < MC; ++k) u = cfma(a[i][k], vc[k], u);
        v[2 * i] = u.x;
        v[2 * i + 1] = u.y;
    }
    if constexpr (WY) {
        double2 sy = cz();
#pragma unroll
        for (int k = K0; k < MC; ++k) sy = cfma(y[k], vc[k], sy);
        v[2 * MR] = sy.x;
        v[2 * MR + 1] = sy.y;
    }
    rowsum_many<P, Q, CS, NV>(v);
#pragma unroll
    for (int i = 0; i < MR; ++i) {
        const double2 u = make_double2(v[2 * i], v[2 * i + 1]);
#pragma unroll
        for (int k = K0; k < MC; ++k) a[i][k] = cfms_cb(u, vc[k], a[i][k]);
    }
    if constexpr (WY) {
        const double2 sy = make_double2(v[2 * MR], v[2 * MR + 1]);
#pragma unroll
        for (int k = K0; k < MC; ++k) y[k] = cfms_cb(sy, vc[k], y[k]);
    }
}

template <int P, bool CS>
__device__ __forceinline__ double2 csum_cols(double2 a) {
    return make_double2(sum_cols<P, CS>(a.x), sum_cols<P, CS>(a.y));
}

// 1/sqrt(x), x > 0: hardware estimate and two Newton steps (full FP64 accuracy).
__device__ __forceinline__ double rsq_nr(double x) {
    double y = __builtin_amdgcn_rsq(x);
    const double h = 0.5 * x;
    y = y * fma(-h * y, y, 1.5);
    y = y * fma(-h * y, y, 1.5);
    return y;
}

// Householder reflector P = I - v v^H (|v|^2 = 2) with P x = -phase |x| e_1,
// phase = x0 / |x0| (1 for x0 = 0): from |x|^2 and the head x0, returns the
// scale of the tail (v_r = x_r scale), the head of v and the new subdiagonal
// entry.  |x| = 0 gives v = 0.
// With t = |x| / |x0| = |x|^2 / sqrt(|x0|^2 |x|^2):  |v|^2 / 2 before scaling is
// |x|^2 + |x0| |x| = |x|^2 + |x0|^2 t,  v_0 = x0 (1 + t) scale  and the new
// subdiagonal -phase |x| = -x0 t: two reciprocal square roots.  Products
// |x0|^2 |x|^2 outside the normal range take the three-root form below.
__device__ __forceinline__ void householder(double norm2, double2 x0, double& scale, double2& vhead,
                                            double2& newsub) {
    const double ax2 = cabs2(x0);
    const double p = ax2 * norm2;
    if (p >= 0x1p-1022 && p <= 0x1p1022) {
        const double t = norm2 * rsq_nr(p);
        scale = rsq_nr(fma(ax2, t, norm2));
        vhead = cscale(x0, (1.0 + t) * scale);
        newsub = cscale(x0, -t);
    } else if (norm2 > 0.0) {
        const double xnorm = norm2 * rsq_nr(norm2);
        double2 phase = make_double2(1.0, 0.0);
        double ax0 = 0.0;
        if (ax2 > 0.0) {
            const double ra = rsq_nr(ax2);
            ax0 = ax2 * ra;
            phase = cscale(x0, ra);
        }
        scale = rsq_nr(fma(ax0, xnorm, norm2));
        vhead = cscale(phase, (ax0 + xnorm) * scale);
        newsub = cscale(phase, -xnorm);
    } else {
        scale = 0.0;
        vhead = cz();
        newsub = cz();
    }
}

// ---- La Budde number type: double2 (FP64 path) or float2 (FP32 path) ----

template <class V> struct CxT;
template <> struct CxT<double2> { using S = double; };
template <> struct CxT<float2> { using S = float; };

template <class V> __device__ __forceinline__ V vmk(typename CxT<V>::S x, typename CxT<V>::S y) {
    V r;
    r.x = x;
    r.y = y;
    return r;
}
template <class V> __device__ __forceinline__ V vzero() { return vmk<V>(0, 0); }
template <class V> __device__ __forceinline__ V vone() { return vmk<V>(1, 0); }
template <class V> __device__ __forceinline__ V vconv(double2 z) {
    return vmk<V>((typename CxT<V>::S)z.x, (typename CxT<V>::S)z.y);
}
template <class V> __device__ __forceinline__ V vmul(V a, V b) {
    return vmk<V>(fma(a.x, b.x, -a.y * b.y), fma(a.x, b.y, a.y * b.x));
}
// c - a * b
template <class V> __device__ __forceinline__ V vfms(V a, V b, V c) {
    return vmk<V>(fma(-a.x, b.x, fma(a.y, b.y, c.x)), fma(-a.x, b.y, fma(-a.y, b.x, c.y)));
}
__device__ __forceinline__ double shr1(double x) { return dpp_mov<0x138>(x); }  // wave_shr:1
__device__ __forceinline__ float shr1(float x) {
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(x), 0x138, 0xF, 0xF, false));
}
__device__ __forceinline__ float swap_sum32(float x) {
    auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(x), __float_as_uint(x), false, false);
    return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}

struct Lds {
    double2* vbuf;   // [W][64]: source column of the current reflector (Hessenberg phase)
    double2* misc;   // [W][2]: squared norm, alpha (border subdiagonal)
    int* idx;        // [W][64]: vertex indices of the subset (gather phase)
    double2* rowbuf; // [NT][RB]: current row of H' (La Budde)
    void* betab;     // [NT][D + 1]: beta_k of the current row (La Budde type)
    void* ring;      // [NT][RS * RS]: last RS trailing characteristic polynomials (anti-diagonal rows)
};

// Row-buffer length per La Budde team: the register tile of a row spans at
// most m + Q - 1 <= 2D + 5 entries (m <= 2n = 2D - 2, Q <= 8).
__host__ __device__ constexpr int lds_rowbuf_len(int D) { return (2 * D + 9 >= 64) ? 64 : ((2 * D + 9) & ~3); }

// Per-wave LDS layout in bytes: misc, rowbuf, betab, then one region that the
// gather / Hessenberg phase uses for vbuf and idx and La Budde then reuses for
// the ring (the phases are separated by a wave-level fence).
struct LdsLayout {
    size_t rowbuf, betab, region, total;
};
__host__ __device__ constexpr LdsLayout lds_layout(int W, int T, int D, int vbytes) {
    const size_t NT = (size_t)(64 / T), RS = (size_t)(D + 1);
    const size_t rowbuf = (size_t)16 * W * 2;
    const size_t betab = rowbuf + (size_t)16 * NT * lds_rowbuf_len(D);
    const size_t region = (betab + (size_t)vbytes * NT * RS + 15) & ~(size_t)15;
    const size_t ring_b = (size_t)vbytes * NT * RS * RS, hess_b = (size_t)(16 + 4) * W * 64;
    return LdsLayout{rowbuf, betab, region, (region + (ring_b > hess_b ? ring_b : hess_b) + 15) & ~(size_t)15};
}

// La Budde team layout: teams of T lanes (P Q, or 64 when a subset needs more
// than P Q coefficient lanes).  Within a team, coefficient d gets a group of
// g_d lanes (a power of two, at most 4) that split its terms k = 1..d-1; the
// lane map (d, g_d, first k, last k) per team lane is a table built on the host
// for every (T, D), so the longest lane carries about D^2 / (2 T) terms instead
// of D - 1.
__host__ __device__ constexpr int lb_team(int G, int D) { return (G >= D + 1) ? G : 64; }
// Team variant of a launch: 0 = teams of P Q lanes, 1 = one team of 64 lanes.
__host__ __device__ constexpr int lb_variant(int G, int D) { return (lb_team(G, D) < 64) ? 0 : 1; }
constexpr int kLbMaxD = kMaxPairs + 2;  // D = n + 1 <= 33
// Offset (in int4 entries) of the lane map of teams of T lanes for D.
__host__ __device__ constexpr int lb_table_offset(int T, int D) {
    return (((T == 16) ? 0 : (T == 32) ? 1 : 2) * kLbMaxD + D) * 64;
}

// LDS bytes of the per-subset kernel with teams of T lanes (64 / T teams);
// vbytes = size of the La Budde complex type.  Non-decreasing in D.
__host__ __device__ constexpr size_t charpoly_lds_bytes(int W, int T, int D, int vbytes) {
    return lds_layout(W, T, D, vbytes).total;
}

// Hessenberg reduction of the tile holding C at rows and columns O .. O+m-1
// (indices below O are zero padding): reflector j (a tile index) zeroes
// column j below row j + 1, for j = O .. O+m-3; phase KJ takes the columns of
// local index KJ.
template <int P, int Q, bool CS, int MR, int MC, int KJ, int O>
__device__ __forceinline__ void hess_phase(double2 (&a)[MR][MC], double2 (&y)[MC], int m, int pr, int pc,
                                           double2* __restrict__ vb) {
    constexpr int IL = (Q * KJ) / P;  // local rows below IL lie above every column of this phase
    constexpr int jj0 = (O > Q * KJ) ? O - Q * KJ : 0;
    for (int jj = jj0; jj < Q; ++jj) {
        const int j = Q * KJ + jj;
        if (j > O + m - 3) return;
        // The lane group holding column j forms the reflector: |x|^2 by a column
        // sum, the head x_{j+1} from the one lane of the group that holds it,
        // then v itself, which it writes for everyone.  With the column-swap map
        // every lane takes the column sums (on its own local column KJ, |x|^2 and
        // the head together) before the group's branch, so the swaps run on the
        // whole wavefront.
        double2 newsub = cz();
        double norm2 = 0.0;
        double2 x0 = cz();
        wave_sync();
        if constexpr (CS) {
            double part = 0.0;
            double2 head = cz();
#pragma unroll
            for (int i = IL; i < MR; ++i) {
                const int r = pr + P * i;
                const double2 x = (r >= j + 1) ? a[i][KJ] : cz();
                part += cabs2(x);
                if (r == j + 1) head = x;
            }
            double sv[4] = {part, head.x, head.y, 0.0};
            colsum_many<P, CS, 4>(sv);
            norm2 = sv[0];
            x0 = make_double2(sv[1], sv[2]);
        }
        if (pc == jj) {
            if constexpr (!CS) {
                double part = 0.0;
                double2 head = cz();
#pragma unroll
                for (int i = IL; i < MR; ++i) {
                    const int r = pr + P * i;
                    const double2 x = (r >= j + 1) ? a[i][KJ] : cz();
                    part += cabs2(x);
                    if (r == j + 1) head = x;
                }
                norm2 = sum_cols<P, CS>(part);
                // the head is in lane P jj + (j + 1) mod P of the group: with one
                // group per wavefront it is read from there, cheaper than a column
                // sum of the others' zeros (with two groups, two reads and a
                // select are not)
                if constexpr (P * Q == 64)
                    x0 = readlane_c(head, P * jj + (j + 1) % P);
                else
                    x0 = csum_cols<P, CS>(head);
            }
            double scale;
            double2 vhead;
            householder(norm2, x0, scale, vhead, newsub);
#pragma unroll
            for (int i = IL; i < MR; ++i) {
                const int r = pr + P * i;
                const double2 x = (r >= j + 1) ? a[i][KJ] : cz();
                vb[r] = (r == j + 1) ? vhead : cscale(x, scale);
            }
        }
        wave_sync();
        double2 vr[MR], vc[MC];
#pragma unroll
        for (int i = IL; i < MR; ++i) vr[i] = vb[pr + P * i];
#pragma unroll
        for (int k = KJ; k < MC; ++k) vc[k] = vb[pc + Q * k];
        // left: H <- (I - v v^H) H
        left_apply<P, CS, MR, MC, IL, KJ>(a, vr);
        if (pc == jj) {
#pragma unroll
            for (int i = IL; i < MR; ++i) {
                const int r = pr + P * i;
                if (r == j + 1) a[i][KJ] = newsub;
                else if (r > j + 1) a[i][KJ] = cz();
            }
        }
        // right: H <- H (I - v v^H); border row y^T <- y^T (I - v v^H)
        right_apply<P, Q, CS, MR, MC, KJ, (O == 0)>(a, y, vc);
    }
}

template <int P, int Q, bool CS, int MR, int MC, int KJ, int O>
__device__ __forceinline__ void hess_all(double2 (&a)[MR][MC], double2 (&y)[MC], int m, int pr, int pc,
                                         double2* __restrict__ vb) {
    if constexpr (KJ < MC) {
        if constexpr (Q * KJ + Q <= O) {  // the phase lies wholly in the padding
            hess_all<P, Q, CS, MR, MC, KJ + 1, O>(a, y, m, pr, pc, vb);
            return;
        }
        if (Q * KJ > O + m - 3) return;
        hess_phase<P, Q, CS, MR, MC, KJ, O>(a, y, m, pr, pc, vb);
        hess_all<P, Q, CS, MR, MC, KJ + 1, O>(a, y, m, pr, pc, vb);
    }
}

// Terms of the La Budde sum loaded per batch: the ring and beta reads of a
// batch are all issued before its first multiply-add, so one LDS latency is
// exposed per batch instead of one per term (the sum keeps its order).
constexpr int kLbBatch = 2;

// One La Budde step (team-local): row r = rho + 1 of H' is in rowbuf at
// index rho + k for H'[r][r + k]; sub_in = H'[r + 1][r].  Team lane tl keeps
// pi_{r,tl} and writes beta_{tl}; under the lane map mp = (d, g, klo, khi) it
// sums the terms klo..khi of coefficient d; the group's partial sums are added
// across its lanes and the first lane stores coefficient d.  gmax: the largest
// group of the team (the same in every lane).  row = (r + d) mod (D + 1), the
// ring row of the lane's coefficient, and rowoff = row (D + 1), kept by the
// caller (both step down by one row per step: no division or multiply here).
template <class V>
__device__ __forceinline__ void labudde_step(int rho, int m, int D, int tl, int4 mp, int gmax,
                                             typename CxT<V>::S m1, typename CxT<V>::S m2, V hrr, V sub_in, V& pik,
                                             const double2* __restrict__ rowbuf, V* __restrict__ betab,
                                             V* __restrict__ ring, int row, int rowoff) {
    const int RS = D + 1;
    // pi_{r,k} = H'[r+1][r] pi_{r+1,k-1} (lane shift by one), pi_{r,0} = 1
    const V sh = vmk<V>(shr1(pik.x), shr1(pik.y));
    pik = (tl == 0) ? vone<V>() : vmul(sub_in, sh);
    const int K = min(D - 1, m - rho - 1);
    if (tl >= 1 && tl <= K) betab[tl] = vmul(vconv<V>(rowbuf[rho + tl]), pik);
    wave_sync();
    // Ring layout: coefficient c of the trailing polynomial of row u is stored at
    // ring[((u + c) % RS) RS + c].  Every term of coefficient d in this step reads
    // coefficient d - k - 1 of row r + k + 1, i.e. the same ring row (r + d) % RS,
    // walking down its columns; no slot wraps inside the k loop.
    const int d = mp.x;
    const bool lead = (tl & (mp.y - 1)) == 0;
    V e = vzero<V>();
    if (d >= 0) {
        if (lead) {
            const int rowpoff = (row + 1 == RS) ? 0 : rowoff + RS;
            e = ring[rowpoff + d];
            if (d >= 1) e = vfms(hrr, ring[rowoff + d - 1], e);
        }
        const int nt = min(mp.w, min(K, d - 1)) - mp.z + 1;  // terms of this lane (may be <= 0)
        const V* rp = ring + rowoff + d - 1 - mp.z;
        const V* bp = betab + mp.z;
        int k0 = 0;
        for (; k0 + kLbBatch <= nt; k0 += kLbBatch) {
            V bv[kLbBatch], rv[kLbBatch];
#pragma unroll
            for (int q = 0; q < kLbBatch; ++q) {
                bv[q] = bp[k0 + q];
                rv[q] = rp[-(k0 + q)];
            }
#pragma unroll
            for (int q = 0; q < kLbBatch; ++q) e = vfms(bv[q], rv[q], e);
        }
        for (; k0 < nt; ++k0) e = vfms(bp[k0], rp[-k0], e);
    }
    // group sums: groups are aligned blocks of 1, 2 or 4 lanes; m1 = 1 in groups
    // of 2 or more, m2 = 1 in groups of 4, else 0 (butterfly over lane ^ 1, ^ 2)
    if (gmax > 1) {
        e = vmk<V>(fma(m1, dpp_mov<0xB1>(e.x), e.x), fma(m1, dpp_mov<0xB1>(e.y), e.y));
        if (gmax > 2) e = vmk<V>(fma(m2, dpp_mov<0x4E>(e.x), e.x), fma(m2, dpp_mov<0x4E>(e.y), e.y));
    }
    if (lead && d >= 0) ring[rowoff + d] = e;
    wave_sync();
}

// Rows of the tile are read bottom-up into rowbuf_own at their tile column
// indices; C sits at tile offset O, so rowbuf (already advanced by O) holds the
// row in C's own column indices and rho is C's row index.
template <int P, int Q, int MR, int MC, int I, class V, int O>
__device__ __forceinline__ void labudde_rows(const double2 (&a)[MR][MC], int m, int D, int tl, int4 mp, int gmax,
                                             typename CxT<V>::S m1, typename CxT<V>::S m2, int pr, int pc,
                                             bool row_owner_group, double2* __restrict__ rowbuf_own,
                                             const double2* __restrict__ rowbuf, V* __restrict__ betab,
                                             V* __restrict__ ring, V& pik, V& sub, int& row, int& rowoff) {
    if constexpr (I >= 0) {
        for (int p = P - 1; p >= 0; --p) {
            const int rho = p + P * I - O;
            if (rho >= m || rho < 0) continue;
            if (row_owner_group && pr == p) {
#pragma unroll
                for (int k = 0; k < MC; ++k) rowbuf_own[pc + Q * k] = a[I][k];
            }
            wave_sync();
            const V hrr = vconv<V>(rowbuf[rho]);
            const V sub_next = (rho >= 1) ? vconv<V>(rowbuf[rho - 1]) : vzero<V>();
            labudde_step<V>(rho, m, D, tl, mp, gmax, m1, m2, hrr, sub, pik, rowbuf, betab, ring, row, rowoff);
            sub = sub_next;
            // (r + d) mod (D + 1) for the next r = rho, and its ring offset
            rowoff = (row == 0) ? D * (D + 1) : rowoff - (D + 1);
            row = (row == 0) ? D : row - 1;
        }
        labudde_rows<P, Q, MR, MC, I - 1, V, O>(a, m, D, tl, mp, gmax, m1, m2, pr, pc, row_owner_group, rowbuf_own,
                                                rowbuf, betab, ring, pik, sub, row, rowoff);
    }
}

// One wavefront's work: the W subsets with local indices first .. first+W-1
// of a run of `count` subsets of size s (colex ranks rank0 + index, or the
// explicit masks), each written to Eout + index * 2(D+1).
// V: complex type of the La Budde recurrence and of the output (double2 for
// the FP64 path, float2 for the FP32 path; the Hessenberg reduction is FP64).
// La Budde teams have TEAM lanes (P Q, or 64 when a subset needs more than
// P Q coefficient lanes), fixed per launch; lbm is the lane map of (TEAM, D).
// LOOPED: the caller runs this in a loop (persistent kernels).  The lane index
// is then passed through an empty asm statement, so the compiler cannot hoist
// the lane-dependent index and predicate arithmetic of the body out of the
// loop and keep it live across iterations (that costs 40-70 VGPRs and
// halves the occupancy of the persistent kernels).
template <int P, int Q, int MR, int MC, class V, int TEAM, int O = 0, bool LOOPED = false>
__device__ __forceinline__ void charpoly_wave(const double2* __restrict__ A0, const double2* __restrict__ dvec, int Np,
                                              int s, uint64_t rank0, uint64_t count, uint64_t first,
                                              const uint64_t* __restrict__ masks, const uint64_t* __restrict__ binom,
                                              int D, const int4* __restrict__ lbm, V* __restrict__ Eout,
                                              double2* __restrict__ lds, uint64_t& chain) {
    constexpr int T = TEAM;
    constexpr int G = P * Q;
    constexpr int W = 64 / G;
    int lane = threadIdx.x;
    if constexpr (LOOPED) asm volatile("" : "+v"(lane));
    constexpr bool CS = lane_map_cs<P, Q, MR, MC, TEAM, O>();
    const int g = LaneMap<P, Q, CS>::g(lane);
    const int pr = LaneMap<P, Q, CS>::pr(lane);
    const int pc = LaneMap<P, Q, CS>::pc(lane);
    const int gl = pc * P + pr;  // lane index within the group
    const int n = Np >> 1;
    const int m = 2 * s;
    constexpr int NT = 64 / T;
    const int RS = D + 1;
    Lds L;
    const LdsLayout ly = lds_layout(W, T, D, (int)sizeof(V));
    const int RB = lds_rowbuf_len(D);
    char* lbase = reinterpret_cast<char*>(lds);
    L.misc = lds;
    L.rowbuf = reinterpret_cast<double2*>(lbase + ly.rowbuf);
    L.betab = lbase + ly.betab;
    L.ring = lbase + ly.region;
    L.vbuf = reinterpret_cast<double2*>(lbase + ly.region);
    L.idx = reinterpret_cast<int*>(lbase + ly.region + (size_t)16 * W * 64);
    double2* vb = L.vbuf + g * 64;
    double2* nb = L.misc + g * 2;
    int* idx = L.idx + g * 64;

    // subsets of this wave (one per group), on the scalar unit: the mask list,
    // or the colex successor of the previous subset (`chain`: the last subset
    // of the caller's previous wave over consecutive ranks, 0 for none, when
    // the first rank is unranked); groups past the end repeat the last subset.
    // Selected per lane; chain returns this wave's last subset.
    uint64_t mask = 0;
    {
        uint64_t mq = masks ? masks[first] : (chain ? colex_next(chain) : unrank_colex(rank0 + first, n, s, binom));
#pragma unroll
        for (int q = 0; q < W; ++q) {
            if (g == q) mask = mq;
            if (q + 1 < W && first + q + 1 < count) mq = masks ? masks[first + q + 1] : colex_next(mq);
        }
        chain = mq;
    }
    for (int e = lane; e < W * 64; e += 64) L.vbuf[e] = cz();
    {
        const int b = gl;  // each group lane b < n scans vertex b
        if (b < n && ((mask >> b) & 1ull)) {
            const int pos = __popcll(mask & ((1ull << b) - 1ull));
            idx[pos] = b;
            idx[pos + s] = b + n;
        }
        if (G < 32) {  // groups narrower than n: lanes scan vertices b + G, b + 2G, ...
            for (int bb = b + G; bb < n; bb += G) {
                if ((mask >> bb) & 1ull) {
                    const int pos = __popcll(mask & ((1ull << bb) - 1ull));
                    idx[pos] = bb;
                    idx[pos + s] = bb + n;
                }
            }
        }
    }
    wave_sync();

    // gather C = X_S A0_S, border row y = d_S and border column z = X_S d_S.
    // C occupies tile rows and columns O .. O+m-1 of the P MR x Q MC tile
    // (O + m <= min(P MR, Q MC)); zero padding in front is passed by the
    // reflectors of the first phase and dropped by later phases with their
    // local index.
    constexpr int o = O;
    double2 a[MR][MC];
    double2 y[MC];
    double2 zr[MR], zc[MC];
#pragma unroll
    for (int i = 0; i < MR; ++i) {
        const int r = pr + P * i - o;
        const bool rok = r >= 0 && r < m;
        const int xr = (r < s) ? r + s : r - s;
        const int vr = rok ? idx[xr] : 0;
        zr[i] = rok ? dvec[vr] : cz();
#pragma unroll
        for (int k = 0; k < MC; ++k) {
            const int c = pc + Q * k - o;
            const bool ok = rok && c >= 0 && c < m;
            const int off = ok ? vr * Np + idx[c] : 0;
            const double2 v = A0[off];
            a[i][k] = ok ? v : cz();
        }
    }
#pragma unroll
    for (int k = 0; k < MC; ++k) {
        const int c = pc + Q * k - o;
        const bool ok = c >= 0 && c < m;
        const int xc = (c < s) ? c + s : c - s;
        const double2 dy = dvec[ok ? idx[c] : 0];
        const double2 dz = dvec[ok ? idx[xc] : 0];
        y[k] = ok ? dy : cz();
        // with spare rows in front, the border row lives in tile row O - 1
        if constexpr (O >= 1)
            if (pr == (O - 1) % P) a[(O - 1) / P][k] = y[k];
        zc[k] = ok ? dz : cz();
    }

    // border reflector: maps z to alpha e_1, applied to C from both sides
    double2 alpha;
    {
        double part = 0.0;
#pragma unroll
        for (int i = 0; i < MR; ++i) part += cabs2(zr[i]);
        const double norm2 = sum_cols<P, CS>(part);
        const double2 x0 = dvec[idx[s]];  // z_0 = loop weight of the partner of vertex 0
        double scale;
        double2 vhead;
        householder(norm2, x0, scale, vhead, alpha);
        double2 vr[MR], vc[MC];
#pragma unroll
        for (int i = 0; i < MR; ++i) vr[i] = (pr + P * i == o) ? vhead : cscale(zr[i], scale);
#pragma unroll
        for (int k = 0; k < MC; ++k) vc[k] = (pc + Q * k == o) ? vhead : cscale(zc[k], scale);
        left_apply<P, CS, MR, MC, 0, 0>(a, vr);
        right_apply<P, Q, CS, MR, MC, 0, (O == 0)>(a, y, vc);
    }
    if (gl == 0) nb[1] = alpha;

    // Householder reduction of the C block
    hess_all<P, Q, CS, MR, MC, 0, O>(a, y, m, pr, pc, vb);
    // vbuf and idx are dead from here on; the La Budde ring reuses their space
    wave_sync();

    // La Budde over the trailing blocks of H' (size m + 1).  Team t of T lanes
    // handles group t + NT * pass; lane d of the team holds coefficient d.
    const int team = lane / T;
    const int tl = lane % T;
    const int4 mp = lbm[tl];
    const int gmax = __builtin_amdgcn_readfirstlane(mp.y);  // team lane 0 leads the largest group
    using S = typename CxT<V>::S;
    const S m1 = (mp.y >= 2) ? (S)1 : (S)0;
    const S m2 = (mp.y >= 4) ? (S)1 : (S)0;
    const int Mp = m + 1;
    for (int pass = 0; pass < W / NT; ++pass) {
        const int gt = pass * NT + team;          // group served by my team
        const bool own = (g / NT) == pass;        // my group's rows are read this pass
        double2* rowbuf_own = L.rowbuf + (g % NT) * RB;
        const double2* rowbuf = L.rowbuf + team * RB + o;  // C's column 0
        V* betab = reinterpret_cast<V*>(L.betab) + team * RS;
        V* ring = reinterpret_cast<V*>(L.ring) + team * RS * RS;
        if (tl < RS) ring[((Mp + tl) % RS) * RS + tl] = (tl == 0) ? vone<V>() : vzero<V>();
        V pik = (tl == 0) ? vone<V>() : vzero<V>();
        V sub = vzero<V>();
        // ring row of the lane's coefficient for the first step (r = m); idle
        // lanes (d = -1) carry a row they never use
        int row = (m + max(mp.x, 0)) % RS;
        int rowoff = row * RS;
        wave_sync();
        labudde_rows<P, Q, MR, MC, MR - 1, V, O>(a, m, D, tl, mp, gmax, m1, m2, pr, pc, own, rowbuf_own, rowbuf,
                                                 betab, ring, pik, sub, row, rowoff);
        // border row: H'[0][k] = y''_{k-1}, H'[0][0] = 0, H'[1][0] = alpha (in y, or
        // in tile row O - 1 when the tile has spare rows in front)
        if (own && pr == ((O >= 1) ? (O - 1) % P : 0)) {
#pragma unroll
            for (int k = 0; k < MC; ++k) rowbuf_own[pc + Q * k] = (O >= 1) ? a[(O - 1) / P][k] : y[k];
        }
        wave_sync();
        const V alpha_t = vconv<V>(L.misc[gt * 2 + 1]);
        labudde_step<V>(-1, m, D, tl, mp, gmax, m1, m2, vzero<V>(), alpha_t, pik, rowbuf, betab, ring, row, rowoff);
        const uint64_t gi = first + gt;
        if (tl <= D && gi < count) {
            V* out = Eout + gi * (uint64_t)(2 * RS);
            out[tl] = ring[((1 + tl) % RS) * RS + tl];  // row 1: det(xI - C)
            out[RS + tl] = ring[tl * RS + tl];          // row 0: det(xI - C')
        }
        wave_sync();
    }
}


template <int P, int Q, int MR, int MC, class V, int TEAM, int O>
__global__ void __launch_bounds__(64, (charpoly_min_waves<P, Q, MR, MC, V, TEAM, O>()))
    charpoly_kernel(const double2* __restrict__ A0, const double2* __restrict__ dvec, int Np, int s, uint64_t rank0,
                    uint64_t count, const uint64_t* __restrict__ masks, const uint64_t* __restrict__ binom, int D,
                    const int4* __restrict__ lbm, V* __restrict__ Eout) {
    extern __shared__ double2 lds[];
    constexpr int W = 64 / (P * Q);
    uint64_t chain = 0;
    charpoly_wave<P, Q, MR, MC, V, TEAM, O>(A0, dvec, Np, s, rank0, count, (uint64_t)blockIdx.x * W, masks, binom, D,
                                            lbm, Eout, lds, chain);
}

// Persistent form for batches: every wavefront takes tiles from `tiles`
// (largest first) through a device counter until none is left, and runs all
// subsets of each tile.  The counter is cleared by the caller's fill kernel.
// All tiles of a launch have C at tile offset O.
template <int P, int Q, int MR, int MC, class V, int TEAM, int O>
__global__ void __launch_bounds__(64) charpoly_batch_kernel(const BatchTile* __restrict__ tiles, int ntiles,
                                                            const BatchItem* __restrict__ items,
                                                            const uint64_t* __restrict__ binom,
                                                            const int4* __restrict__ lbmap,
                                                            unsigned* __restrict__ counter, V* __restrict__ Ebase) {
    extern __shared__ double2 lds[];
    constexpr int G = P * Q;
    constexpr int W = 64 / G;
    for (;;) {
        int t = 0;
        if (threadIdx.x == 0) t = (int)atomicAdd(counter, 1u);
        // readfirstlane keeps the tile index, and everything loaded from the
        // tile and item records, in scalar registers
        t = __builtin_amdgcn_readfirstlane(t);
        if (t >= ntiles) break;
        const BatchTile tl = tiles[t];
        const BatchItem it = items[tl.item];
        const int D = it.n + 1;
        if (TEAM < D + 1) continue;  // a team must hold D + 1 coefficients; the plan never sends such tiles
        const int4* lbm = lbmap + lb_table_offset(TEAM, D);
        uint64_t chain = 0;
        for (uint64_t first = 0; first < tl.count; first += W)
            charpoly_wave<P, Q, MR, MC, V, TEAM, O, true>(it.A0, it.dvec, it.Np, tl.s, tl.rank0, tl.count, first,
                                                          nullptr, binom, D, lbm, Ebase + tl.eoff, lds, chain);
        wave_sync();
    }
}

}  // namespace gbs
