// HIP kernels (gfx950 / CDNA4) for the loop-hafnian power-trace subset sum.
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
// Register layout of the m x m Hessenberg work (one wavefront per subset):
// lane = pr + 8 pc (pr, pc in 0..7); lane owns rows r = pr + 8 i and columns
// c = pc + 8 k, i, k < MB, MB = ceil(m / 8).  Column sums reduce over the 8
// lanes of an octet (DPP), row sums over the 8 lanes of stride 8 (DPP row_ror
// plus the gfx950 permlane16/32 swaps).

#include <hip/hip_runtime.h>
#include <stdint.h>

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

// ---------------------------------------------------------------- phase 1

struct WaveLds {
    double2* vbuf;   // 64: current reflector source column
    double2* rowbuf; // 64: current row of H' for La Budde
    double2* betab;  // 64: La Budde coefficients beta_k of the current row
    double2* ring;   // RS x RS: last RS trailing characteristic polynomials
    int* idx;        // 64: vertex indices of the subset
};

__host__ __device__ constexpr int wave_lds_doubles2(int D) { return 192 + (D + 1) * (D + 1) + 16; }

template <int MB, int KJ>
__device__ __forceinline__ void hess_phase(double2 (&a)[MB][MB], double2 (&y)[MB], int m, int pr, int pc,
                                           const WaveLds& L) {
    for (int jj = 0; jj < 8; ++jj) {
        const int j = 8 * KJ + jj;
        if (j > m - 3) return;
        wave_sync();
        // squared norm of the column below the diagonal (owner octet pc == jj)
        double part = 0.0;
#pragma unroll
        for (int i = KJ; i < MB; ++i) {
            const int r = pr + 8 * i;
            if (r >= j + 1) part += cabs2(a[i][KJ]);
        }
        part = sum_octet(part);
        const double norm2 = readlane_d(part, 8 * jj);
        // x0 = H[j+1][j] sits in lane ((j+1)&7) + 8 jj at local row (j+1)>>3
        constexpr int KN = (KJ + 1 < MB) ? KJ + 1 : KJ;
        const double2 cand = (((j + 1) >> 3) == KJ) ? a[KJ][KJ] : a[KN][KJ];
        const double2 x0 = readlane_c(cand, ((j + 1) & 7) + 8 * jj);
        if (pc == jj) {
#pragma unroll
            for (int i = KJ; i < MB; ++i) {
                const int r = pr + 8 * i;
                L.vbuf[r] = (r >= j + 1) ? a[i][KJ] : cz();
            }
        }
        wave_sync();
        if (norm2 == 0.0) continue;  // column already reduced: identity reflector
        const double xnorm = sqrt(norm2);
        const double ax0 = sqrt(cabs2(x0));
        const double2 phase = (ax0 == 0.0) ? make_double2(1.0, 0.0) : cscale(x0, 1.0 / ax0);
        const double scale = 1.0 / sqrt(fma(ax0, xnorm, norm2));
        const double2 vhead = cscale(phase, (ax0 + xnorm) * scale);
        const double2 newsub = cscale(phase, -xnorm);
        double2 vr[MB], vc[MB];
#pragma unroll
        for (int i = KJ; i < MB; ++i) {
            const int r = pr + 8 * i;
            vr[i] = (r == j + 1) ? vhead : cscale(L.vbuf[r], scale);
        }
#pragma unroll
        for (int k = KJ; k < MB; ++k) {
            const int c = pc + 8 * k;
            vc[k] = (c == j + 1) ? vhead : cscale(L.vbuf[c], scale);
        }
        // left: H <- (I - v v^H) H on rows > j
#pragma unroll
        for (int k = KJ; k < MB; ++k) {
            double2 w = cz();
#pragma unroll
            for (int i = KJ; i < MB; ++i) w = cfma_ca(vr[i], a[i][k], w);
            w = csum_octet(w);
#pragma unroll
            for (int i = KJ; i < MB; ++i) a[i][k] = cfms(vr[i], w, a[i][k]);
        }
        // column j becomes exactly (.., newsub, 0, .., 0)^T
        if (pc == jj) {
#pragma unroll
            for (int i = KJ; i < MB; ++i) {
                const int r = pr + 8 * i;
                if (r == j + 1) a[i][KJ] = newsub;
                else if (r > j + 1) a[i][KJ] = cz();
            }
        }
        // right: H <- H (I - v v^H) on columns > j, all rows
#pragma unroll
        for (int i = 0; i < MB; ++i) {
            double2 u = cz();
#pragma unroll
            for (int k = KJ; k < MB; ++k) u = cfma(a[i][k], vc[k], u);
            u = csum_stride8(u);
#pragma unroll
            for (int k = KJ; k < MB; ++k) a[i][k] = cfms_cb(u, vc[k], a[i][k]);
        }
        // border row y^T <- y^T (I - v v^H)
        {
            double2 sy = cz();
#pragma unroll
            for (int k = KJ; k < MB; ++k) sy = cfma(y[k], vc[k], sy);
            sy = csum_stride8(sy);
#pragma unroll
            for (int k = KJ; k < MB; ++k) y[k] = cfms_cb(sy, vc[k], y[k]);
        }
    }
}

template <int MB, int KJ>
__device__ __forceinline__ void hess_all(double2 (&a)[MB][MB], double2 (&y)[MB], int m, int pr, int pc,
                                         const WaveLds& L) {
    if constexpr (KJ < MB) {
        if (8 * KJ > m - 3) return;
        hess_phase<MB, KJ>(a, y, m, pr, pc, L);
        hess_all<MB, KJ + 1>(a, y, m, pr, pc, L);
    }
}

// One La Budde step for row r of H' (rho = r - 1 in C coordinates); rowbuf
// holds H'[r][r + k] at index rho + k.  Updates ring slot r.
__device__ __forceinline__ void labudde_step(int rho, int m, int D, int lane, double2 hrr, double2 sub_in,
                                             double2& pik, const WaveLds& L) {
    const int RS = D + 1;
    const int r = rho + 1;
    // pi_{r,k} = H'[r+1][r] * pi_{r+1,k-1}, pi_{r,0} = 1
    double2 sh = make_double2(dpp_mov<0x138>(pik.x), dpp_mov<0x138>(pik.y));  // wave_shr:1
    pik = (lane == 0) ? make_double2(1.0, 0.0) : cmul(sub_in, sh);
    const int K = min(D - 1, m - rho - 1);
    if (lane >= 1 && lane <= K) L.betab[lane] = cmul(L.rowbuf[rho + lane], pik);
    wave_sync();
    if (lane <= D) {
        const double2* prev = L.ring + ((r + 1) % RS) * RS;
        double2 e0 = prev[lane];
        double2 e1 = cz();
        if (lane >= 1) e0 = cfms(hrr, prev[lane - 1], e0);
        // uniform trip count (K), two independent accumulators; lane d only
        // takes terms with k < d (coefficient index d - k - 1 >= 0)
        int slot = (r + 2) % RS;
        int k = 1;
        for (; k + 1 <= K; k += 2) {
            const int s1 = (slot + 1 == RS) ? 0 : slot + 1;
            const double2 b0 = L.betab[k], b1 = L.betab[k + 1];
            const double2 q0 = L.ring[slot * RS + max(lane - k - 1, 0)];
            const double2 q1 = L.ring[s1 * RS + max(lane - k - 2, 0)];
            if (k < lane) e0 = cfms(b0, q0, e0);
            if (k + 1 < lane) e1 = cfms(b1, q1, e1);
            slot = (s1 + 1 == RS) ? 0 : s1 + 1;
        }
        if (k <= K && k < lane) e0 = cfms(L.betab[k], L.ring[slot * RS + lane - k - 1], e0);
        L.ring[(r % RS) * RS + lane] = cadd(e0, e1);
    }
    wave_sync();
}

template <int MB, int I>
__device__ __forceinline__ void labudde_rows(const double2 (&a)[MB][MB], int m, int D, int lane, int pr, int pc,
                                             double2& pik, double2& sub, const WaveLds& L) {
    if constexpr (I >= 0) {
        for (int p = 7; p >= 0; --p) {
            const int rho = p + 8 * I;
            if (rho >= m) continue;
            if (pr == p) {
#pragma unroll
                for (int k = 0; k < MB; ++k) L.rowbuf[pc + 8 * k] = a[I][k];
            }
            wave_sync();
            const double2 hrr = L.rowbuf[rho];
            const double2 sub_next = (rho >= 1) ? L.rowbuf[rho - 1] : cz();
            labudde_step(rho, m, D, lane, hrr, sub, pik, L);
            sub = sub_next;
        }
        labudde_rows<MB, I - 1>(a, m, D, lane, pr, pc, pik, sub, L);
    }
}

template <int MB>
__global__ void __launch_bounds__(64) charpoly_kernel(const double2* __restrict__ A0, const double2* __restrict__ dvec,
                                                      int Np, int s, uint64_t rank0, uint64_t count,
                                                      const uint64_t* __restrict__ masks,
                                                      const uint64_t* __restrict__ binom, int D,
                                                      double2* __restrict__ Eout) {
    extern __shared__ double2 lds[];
    const uint64_t g = blockIdx.x;
    if (g >= count) return;
    const int lane = threadIdx.x;
    const int n = Np >> 1;
    const int m = 2 * s;
    const int pr = lane & 7, pc = lane >> 3;
    const int RS = D + 1;
    WaveLds L;
    L.vbuf = lds;
    L.rowbuf = lds + 64;
    L.betab = lds + 128;
    L.ring = lds + 192;
    L.idx = reinterpret_cast<int*>(lds + 192 + RS * RS);

    const uint64_t mask = masks ? masks[g] : unrank_colex(rank0 + g, n, s, binom);
    if (lane < n && ((mask >> lane) & 1ull)) {
        const int pos = __popcll(mask & ((1ull << lane) - 1ull));
        L.idx[pos] = lane;
        L.idx[pos + s] = lane + n;
    }
    wave_sync();

    // gather C = X_S A0_S, border row y = d_S (columns) and z = X_S d_S
    double2 a[MB][MB];
    double2 y[MB];
    double2 zr[MB], zc[MB];
#pragma unroll
    for (int i = 0; i < MB; ++i) {
        const int r = pr + 8 * i;
        const bool rok = r < m;
        const int xr = (r < s) ? r + s : r - s;
        const int vr = rok ? L.idx[xr] : 0;
        zr[i] = rok ? dvec[vr] : cz();
#pragma unroll
        for (int k = 0; k < MB; ++k) {
            const int c = pc + 8 * k;
            const bool ok = rok && c < m;
            const int off = ok ? vr * Np + L.idx[c] : 0;
            const double2 v = A0[off];
            a[i][k] = ok ? v : cz();
        }
    }
#pragma unroll
    for (int k = 0; k < MB; ++k) {
        const int c = pc + 8 * k;
        const bool ok = c < m;
        const int xc = (c < s) ? c + s : c - s;
        const double2 dy = dvec[ok ? L.idx[c] : 0];
        const double2 dz = dvec[ok ? L.idx[xc] : 0];
        y[k] = ok ? dy : cz();
        zc[k] = ok ? dz : cz();
    }

    // border reflector: maps z to alpha e_1, applied to C from both sides
    double2 alpha = cz();
    {
        double part = 0.0;
#pragma unroll
        for (int i = 0; i < MB; ++i) part += cabs2(zr[i]);
        const double norm2 = sum_octet(part);
        if (norm2 != 0.0) {
            const double2 x0 = dvec[L.idx[s]];  // z_0 = d of the partner of the first vertex
            const double xnorm = sqrt(norm2);
            const double ax0 = sqrt(cabs2(x0));
            const double2 phase = (ax0 == 0.0) ? make_double2(1.0, 0.0) : cscale(x0, 1.0 / ax0);
            const double scale = 1.0 / sqrt(fma(ax0, xnorm, norm2));
            const double2 vhead = cscale(phase, (ax0 + xnorm) * scale);
            alpha = cscale(phase, -xnorm);
            double2 vr[MB], vc[MB];
#pragma unroll
            for (int i = 0; i < MB; ++i) vr[i] = (pr + 8 * i == 0) ? vhead : cscale(zr[i], scale);
#pragma unroll
            for (int k = 0; k < MB; ++k) vc[k] = (pc + 8 * k == 0) ? vhead : cscale(zc[k], scale);
#pragma unroll
            for (int k = 0; k < MB; ++k) {
                double2 w = cz();
#pragma unroll
                for (int i = 0; i < MB; ++i) w = cfma_ca(vr[i], a[i][k], w);
                w = csum_octet(w);
#pragma unroll
                for (int i = 0; i < MB; ++i) a[i][k] = cfms(vr[i], w, a[i][k]);
            }
#pragma unroll
            for (int i = 0; i < MB; ++i) {
                double2 u = cz();
#pragma unroll
                for (int k = 0; k < MB; ++k) u = cfma(a[i][k], vc[k], u);
                u = csum_stride8(u);
#pragma unroll
                for (int k = 0; k < MB; ++k) a[i][k] = cfms_cb(u, vc[k], a[i][k]);
            }
            double2 sy = cz();
#pragma unroll
            for (int k = 0; k < MB; ++k) sy = cfma(y[k], vc[k], sy);
            sy = csum_stride8(sy);
#pragma unroll
            for (int k = 0; k < MB; ++k) y[k] = cfms_cb(sy, vc[k], y[k]);
        }
    }

    // Householder reduction of the C block
    hess_all<MB, 0>(a, y, m, pr, pc, L);

    // La Budde over trailing blocks of H' (size m + 1), bottom row first
    const int Mp = m + 1;
    if (lane < RS) L.ring[(Mp % RS) * RS + lane] = (lane == 0) ? make_double2(1.0, 0.0) : cz();
    double2 pik = (lane == 0) ? make_double2(1.0, 0.0) : cz();
    double2 sub = cz();
    wave_sync();
    labudde_rows<MB, MB - 1>(a, m, D, lane, pr, pc, pik, sub, L);
    // border row: H'[0][k] = y''_{k-1}, H'[0][0] = 0, H'[1][0] = alpha
    if (pr == 0) {
#pragma unroll
        for (int k = 0; k < MB; ++k) L.rowbuf[pc + 8 * k] = y[k];
    }
    wave_sync();
    labudde_step(-1, m, D, lane, cz(), alpha, pik, L);

    // E_1 = det(xI - C) (slot 1), E_0 = det(xI - C') (slot 0): leading D+1 coefficients
    if (lane <= D) {
        double2* out = Eout + g * (uint64_t)(2 * RS);
        out[lane] = L.ring[(1 % RS) * RS + lane];
        out[RS + lane] = L.ring[lane];
    }
}

// ---------------------------------------------------------------- phase 2

__device__ __forceinline__ void two_sum(double a, double b, double& s, double& e) {
    s = a + b;
    const double bb = s - a;
    e = (a - (s - bb)) + (b - bb);
}

struct Acc {
    double sr, cr, si, ci, ab;
};

__device__ __forceinline__ void acc_add(Acc& A, double2 t) {
    double s, e;
    two_sum(A.sr, t.x, s, e);
    A.sr = s;
    A.cr += e;
    two_sum(A.si, t.y, s, e);
    A.si = s;
    A.ci += e;
    A.ab += sqrt(cabs2(t));
}

__device__ __forceinline__ void acc_merge(Acc& A, const Acc& B) {
    double s, e;
    two_sum(A.sr, B.sr, s, e);
    A.sr = s;
    A.cr = A.cr + B.cr + e;
    two_sum(A.si, B.si, s, e);
    A.si = s;
    A.ci = A.ci + B.ci + e;
    A.ab += B.ab;
}

__device__ __forceinline__ double shfl_xor_d(double x, int m) {
    int lo = __shfl_xor(__double2loint(x), m);
    int hi = __shfl_xor(__double2hiint(x), m);
    return __hiloint2double(hi, lo);
}

// Signed term t_S from the leading coefficients of det(xI - C) (R) and
// det(xI - C') (Rp):
//   R(eta) = sum_k R_k eta^k = det(I - eta C)
//   p_k = -k R_k - sum_{j<k} R_j p_{k-j}               (Newton: p_k = tr C^k)
//   L = (R - R') / (eta R):  L_k = (R_{k+1} - R'_{k+1}) - sum_{j<k} R_j L_{k-j}
//   c_k = p_k / (2k) + L_k / 2
//   e_0 = 1, e_k = (1/k) sum_{j<=k} j c_j e_{k-j};  t = sign * e_n
template <int NN>
__device__ __forceinline__ double2 series_term(const double2* __restrict__ E, int RS, double sign) {
    double2 R[NN + 2], c[NN + 1];
#pragma unroll
    for (int k = 0; k <= NN + 1; ++k) R[k] = E[k];
    {
        double2 Lk[NN + 1], p[NN + 1];
        Lk[0] = cz();
#pragma unroll
        for (int k = 1; k <= NN; ++k) {
            double2 acc = csub(R[k + 1], E[RS + k + 1]);
#pragma unroll
            for (int j = 1; j < k; ++j) acc = cfms(R[j], Lk[k - j], acc);
            Lk[k] = acc;
            double2 pk = cscale(R[k], -(double)k);
#pragma unroll
            for (int j = 1; j < k; ++j) pk = cfms(R[j], p[k - j], pk);
            p[k] = pk;
            c[k] = cadd(cscale(pk, 0.5 / k), cscale(acc, 0.5));
        }
    }
    double2 e[NN + 1];
    e[0] = make_double2(1.0, 0.0);
#pragma unroll
    for (int k = 1; k <= NN; ++k) {
        double2 acc = cz();
#pragma unroll
        for (int j = 1; j <= k; ++j) acc = cfma(cscale(c[j], (double)j), e[k - j], acc);
        e[k] = cscale(acc, 1.0 / k);
    }
    return cscale(e[NN], sign);
}

template <int NN>
__global__ void __launch_bounds__(64) series_kernel(const double2* __restrict__ E, uint64_t count, int D,
                                                    double sign, int per_thread, double* __restrict__ partials,
                                                    double2* __restrict__ terms) {
    const int lane = threadIdx.x;
    const int RS = D + 1;
    Acc A{0.0, 0.0, 0.0, 0.0, 0.0};
    const uint64_t base = (uint64_t)blockIdx.x * 64 * per_thread;
    for (int q = 0; q < per_thread; ++q) {
        const uint64_t g = base + (uint64_t)q * 64 + lane;
        if (g < count) {
            const double2 t = series_term<NN>(E + g * (uint64_t)(2 * RS), RS, sign);
            if (terms) terms[g] = t;
            acc_add(A, t);
        }
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        Acc B;
        B.sr = shfl_xor_d(A.sr, off);
        B.cr = shfl_xor_d(A.cr, off);
        B.si = shfl_xor_d(A.si, off);
        B.ci = shfl_xor_d(A.ci, off);
        B.ab = shfl_xor_d(A.ab, off);
        if (lane & off) {
            Acc T = B;
            acc_merge(T, A);
            A = T;
        } else {
            acc_merge(A, B);
        }
    }
    if (lane == 0) {
        double* o = partials + 5 * (uint64_t)blockIdx.x;
        o[0] = A.sr;
        o[1] = A.cr;
        o[2] = A.si;
        o[3] = A.ci;
        o[4] = A.ab;
    }
}

// ---------------------------------------------------------------- reductions / prep

__global__ void __launch_bounds__(256) final_reduce_kernel(const double* __restrict__ partials, int64_t np,
                                                           double2* __restrict__ out,
                                                           double* __restrict__ abs_out) {
    __shared__ double sh[5][256];
    const int t = threadIdx.x;
    Acc A{0.0, 0.0, 0.0, 0.0, 0.0};
    for (int64_t i = t; i < np; i += 256) {
        Acc B{partials[5 * i], partials[5 * i + 1], partials[5 * i + 2], partials[5 * i + 3], partials[5 * i + 4]};
        acc_merge(A, B);
    }
    sh[0][t] = A.sr;
    sh[1][t] = A.cr;
    sh[2][t] = A.si;
    sh[3][t] = A.ci;
    sh[4][t] = A.ab;
    __syncthreads();
    for (int w = 128; w >= 1; w >>= 1) {
        if (t < w) {
            Acc X{sh[0][t], sh[1][t], sh[2][t], sh[3][t], sh[4][t]};
            Acc Y{sh[0][t + w], sh[1][t + w], sh[2][t + w], sh[3][t + w], sh[4][t + w]};
            acc_merge(X, Y);
            sh[0][t] = X.sr;
            sh[1][t] = X.cr;
            sh[2][t] = X.si;
            sh[3][t] = X.ci;
            sh[4][t] = X.ab;
        }
        __syncthreads();
    }
    if (t == 0) {
        out[0] = make_double2(sh[0][0] + sh[1][0], sh[2][0] + sh[3][0]);
        if (abs_out) abs_out[0] = sh[4][0];
    }
}

// A (N x N, leading dim lda) -> A0 (Np x Np, zero diagonal) and d (Np); an odd
// N gets one extra vertex with loop weight 1 and no edges.
__global__ void __launch_bounds__(256) prep_kernel(const double2* __restrict__ A, int N, int64_t lda, int Np,
                                                   double2* __restrict__ A0, double2* __restrict__ d) {
    for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < Np * Np; e += gridDim.x * blockDim.x) {
        const int i = e / Np, j = e % Np;
        double2 v = cz();
        if (i < N && j < N && i != j) v = A[(int64_t)i * lda + j];
        A0[e] = v;
        if (i == j) d[i] = (i < N) ? A[(int64_t)i * lda + i] : make_double2(1.0, 0.0);
    }
}

__global__ void __launch_bounds__(64) scalar_set_kernel(double2* __restrict__ out, double2 v,
                                                        double* __restrict__ abs_out, double a) {
    if (threadIdx.x == 0) {
        out[0] = v;
        if (abs_out) abs_out[0] = a;
    }
}

// Self-check of the cross-lane sums used above: in[64] -> out[4 * 64]
// (octet sums, stride-8 sums, readlane of lane 37, wave_shr:1).
__global__ void __launch_bounds__(64) selftest_kernel(const double* __restrict__ in, double* __restrict__ out) {
    const int l = threadIdx.x;
    const double x = in[l];
    out[l] = sum_octet(x);
    out[64 + l] = sum_stride8(x);
    out[128 + l] = readlane_d(x, 37);
    out[192 + l] = dpp_mov<0x138>(x);
}

// ---------------------------------------------------------------- launchers

template <int MB>
static hipError_t launch_charpoly_mb(const LaunchPhase1& p, hipStream_t st) {
    const size_t lds = sizeof(double2) * wave_lds_doubles2(p.D);
    hipLaunchKernelGGL(charpoly_kernel<MB>, dim3((unsigned)p.count), dim3(64), lds, st, p.A0, p.dvec, p.Np, p.s,
                       p.rank0, p.count, p.masks, p.binom, p.D, p.Eout);
    return hipGetLastError();
}

hipError_t launch_charpoly(const LaunchPhase1& p, hipStream_t st) {
    const int m = 2 * p.s;
    const int MB = (m + 7) / 8;
    switch (MB) {
        case 1: return launch_charpoly_mb<1>(p, st);
        case 2: return launch_charpoly_mb<2>(p, st);
        case 3: return launch_charpoly_mb<3>(p, st);
        case 4: return launch_charpoly_mb<4>(p, st);
        case 5: return launch_charpoly_mb<5>(p, st);
        case 6: return launch_charpoly_mb<6>(p, st);
        case 7: return launch_charpoly_mb<7>(p, st);
        case 8: return launch_charpoly_mb<8>(p, st);
        default: return hipErrorInvalidValue;
    }
}

size_t charpoly_lds_bytes(int D) { return sizeof(double2) * wave_lds_doubles2(D); }

template <int NN>
static hipError_t launch_series_nn(const LaunchPhase2& p, hipStream_t st) {
    const uint64_t per_block = 64ull * p.per_thread;
    const unsigned grid = (unsigned)((p.count + per_block - 1) / per_block);
    hipLaunchKernelGGL(series_kernel<NN>, dim3(grid), dim3(64), 0, st, p.E, p.count, p.D, p.sign, p.per_thread,
                       p.partials, p.terms);
    return hipGetLastError();
}

template <int NN>
static hipError_t series_dispatch(int n, const LaunchPhase2& p, hipStream_t st) {
    if constexpr (NN > kMaxPairs) {
        return hipErrorInvalidValue;
    } else {
        if (n == NN) return launch_series_nn<NN>(p, st);
        return series_dispatch<NN + 1>(n, p, st);
    }
}

hipError_t launch_series(int n, const LaunchPhase2& p, hipStream_t st) { return series_dispatch<1>(n, p, st); }

hipError_t launch_final_reduce(const double* partials, int64_t np, double2* out, double* abs_out, hipStream_t st) {
    hipLaunchKernelGGL(final_reduce_kernel, dim3(1), dim3(256), 0, st, partials, np, out, abs_out);
    return hipGetLastError();
}

hipError_t launch_prep(const double2* A, int N, int64_t lda, int Np, double2* A0, double2* d, hipStream_t st) {
    const int total = Np * Np;
    const int grid = (total + 255) / 256;
    hipLaunchKernelGGL(prep_kernel, dim3(grid > 0 ? grid : 1), dim3(256), 0, st, A, N, lda, Np, A0, d);
    return hipGetLastError();
}

hipError_t launch_scalar_set(double2* out, double2 v, double* abs_out, double a, hipStream_t st) {
    hipLaunchKernelGGL(scalar_set_kernel, dim3(1), dim3(64), 0, st, out, v, abs_out, a);
    return hipGetLastError();
}

hipError_t launch_selftest(const double* in, double* out, hipStream_t st) {
    hipLaunchKernelGGL(selftest_kernel, dim3(1), dim3(64), 0, st, in, out);
    return hipGetLastError();
}

}  // namespace gbs
