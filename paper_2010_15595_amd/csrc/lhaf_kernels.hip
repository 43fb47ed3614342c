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
// Register layout of the m x m Hessenberg work: a wavefront holds W = 64/(P Q)
// subsets of one size class; lane l = g (P Q) + pc P + pr serves subset g and
// owns rows r = pr + P i (i < MR) and columns c = pc + Q k (k < MC).  Column
// sums reduce over the P consecutive lanes (DPP quad_perm / row_half_mirror),
// row sums over the Q lanes of stride P (DPP row_ror plus the gfx950
// permlane16/32 swaps).  Lane grids: 8x8 (one subset per wave), 8x4 (two),
// 4x4 (four); the choice per subset size is made by the host (autotuned).

#include "lhaf_device.h"

namespace gbs {
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
// V is double2 (FP64 path) or float2 (FP32 path).
template <int NN, class V>
__device__ __forceinline__ V series_term(const V* __restrict__ E, int RS, double sign) {
    using S = typename CxT<V>::S;
    V R[NN + 2], c[NN + 1];
#pragma unroll
    for (int k = 0; k <= NN + 1; ++k) R[k] = E[k];
    {
        V Lk[NN + 1], p[NN + 1];
        Lk[0] = vzero<V>();
#pragma unroll
        for (int k = 1; k <= NN; ++k) {
            const V rp = E[RS + k + 1];
            V acc = vmk<V>(R[k + 1].x - rp.x, R[k + 1].y - rp.y);
#pragma unroll
            for (int j = 1; j < k; ++j) acc = vfms(R[j], Lk[k - j], acc);
            Lk[k] = acc;
            V pk = vmk<V>(-(S)k * R[k].x, -(S)k * R[k].y);
#pragma unroll
            for (int j = 1; j < k; ++j) pk = vfms(R[j], p[k - j], pk);
            p[k] = pk;
            const S hk = (S)0.5 / (S)k;
            c[k] = vmk<V>(fma(pk.x, hk, (S)0.5 * acc.x), fma(pk.y, hk, (S)0.5 * acc.y));
        }
    }
    V e[NN + 1];
    e[0] = vone<V>();
#pragma unroll
    for (int k = 1; k <= NN; ++k) {
        V acc = vzero<V>();
#pragma unroll
        for (int j = 1; j <= k; ++j) {
            const V cj = vmk<V>((S)j * c[j].x, (S)j * c[j].y);
            acc = vfms(vmk<V>(-cj.x, -cj.y), e[k - j], acc);
        }
        const S ik = (S)1 / (S)k;
        e[k] = vmk<V>(acc.x * ik, acc.y * ik);
    }
    return vmk<V>(e[NN].x * (S)sign, e[NN].y * (S)sign);
}

template <class S>
__device__ __forceinline__ void two_sum_t(S a, S b, S& s, S& e) {
    s = a + b;
    const S bb = s - a;
    e = (a - (s - bb)) + (b - bb);
}

// One lane per subset.  Each lane accumulates its terms with TwoSum in the
// path's precision (FP32 compensated on the FP32 path); lanes and blocks are
// combined in FP64 in a fixed order.
template <int NN, class V>
__global__ void __launch_bounds__(64) series_kernel(const V* __restrict__ E, uint64_t count, int D, double sign,
                                                    int per_thread, double* __restrict__ partials,
                                                    double2* __restrict__ terms) {
    using S = typename CxT<V>::S;
    const int lane = threadIdx.x;
    const int RS = D + 1;
    S sr = 0, cr = 0, si = 0, ci = 0;
    double ab = 0.0;
    const uint64_t base = (uint64_t)blockIdx.x * 64 * per_thread;
    for (int q = 0; q < per_thread; ++q) {
        const uint64_t g = base + (uint64_t)q * 64 + lane;
        if (g < count) {
            const V t = series_term<NN, V>(E + g * (uint64_t)(2 * RS), RS, sign);
            if (terms) terms[g] = make_double2((double)t.x, (double)t.y);
            S sn, en;
            two_sum_t<S>(sr, t.x, sn, en);
            sr = sn;
            cr += en;
            two_sum_t<S>(si, t.y, sn, en);
            si = sn;
            ci += en;
            ab += sqrt((double)t.x * t.x + (double)t.y * t.y);
        }
    }
    Acc A{(double)sr, (double)cr, (double)si, (double)ci, ab};
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

// Batched series: block b runs up to 64 * per_thread subsets of one tile
// (all tiles of the launch have n = NN pairs).
template <int NN, class V>
__global__ void __launch_bounds__(64) series_batch_kernel(const SeriesBlock* __restrict__ blocks,
                                                          const BatchTile* __restrict__ tiles,
                                                          const V* __restrict__ Ebase, int per_thread,
                                                          double* __restrict__ partials) {
    using S = typename CxT<V>::S;
    const int lane = threadIdx.x;
    const SeriesBlock b = blocks[blockIdx.x];
    const BatchTile tl = tiles[b.tile];
    constexpr int RS = NN + 2;
    const double sign = ((NN - tl.s) & 1) ? -1.0 : 1.0;
    S sr = 0, cr = 0, si = 0, ci = 0;
    double ab = 0.0;
    for (int q = 0; q < per_thread; ++q) {
        const uint64_t g = b.sub0 + (uint64_t)q * 64 + lane;
        if (g < tl.count) {
            const V t = series_term<NN, V>(Ebase + tl.eoff + g * (uint64_t)(2 * RS), RS, sign);
            S sn, en;
            two_sum_t<S>(sr, t.x, sn, en);
            sr = sn;
            cr += en;
            two_sum_t<S>(si, t.y, sn, en);
            si = sn;
            ci += en;
            ab += sqrt((double)t.x * t.x + (double)t.y * t.y);
        }
    }
    Acc A{(double)sr, (double)cr, (double)si, (double)ci, ab};
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
        double* o = partials + 5 * (uint64_t)b.pidx;
        o[0] = A.sr;
        o[1] = A.cr;
        o[2] = A.si;
        o[3] = A.ci;
        o[4] = A.ab;
    }
}

// Per-item fixed-order reduction of partials [pbeg[i], pbeg[i+1]).
__global__ void __launch_bounds__(64) item_reduce_kernel(const int64_t* __restrict__ pbeg,
                                                         const double* __restrict__ partials,
                                                         const BatchItem* __restrict__ items,
                                                         double2* __restrict__ out, double* __restrict__ abs_out) {
    const int i = blockIdx.x;
    const int lane = threadIdx.x;
    // items with pairs but no partials are summed whole by small_items_kernel
    if (pbeg[i + 1] == pbeg[i] && items[i].n > 0) return;
    Acc A{0.0, 0.0, 0.0, 0.0, 0.0};
    for (int64_t k = pbeg[i] + lane; k < pbeg[i + 1]; k += 64) {
        Acc B{partials[5 * k], partials[5 * k + 1], partials[5 * k + 2], partials[5 * k + 3], partials[5 * k + 4]};
        acc_merge(A, B);
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
        const bool empty = pbeg[i + 1] == pbeg[i];  // n = 0: lhaf = 1
        out[i] = empty ? make_double2(1.0, 0.0) : make_double2(A.sr + A.cr, A.si + A.ci);
        if (abs_out) abs_out[i] = empty ? 1.0 : A.ab;
    }
}

// Batch prep: item i (N[i] x N[i] at mats + in_off[i]) -> its A0 and d.
__global__ void __launch_bounds__(256) batch_prep_kernel(const double2* __restrict__ mats,
                                                         const int64_t* __restrict__ in_off,
                                                         const int* __restrict__ Ns,
                                                         const BatchItem* __restrict__ items) {
    const int i = blockIdx.x;
    const BatchItem it = items[i];
    const int N = Ns[i], Np = it.Np;
    const double2* A = mats + in_off[i];
    double2* A0 = const_cast<double2*>(it.A0);
    double2* d = const_cast<double2*>(it.dvec);
    for (int e = threadIdx.x; e < Np * Np; e += blockDim.x) {
        const int r = e / Np, c = e % Np;
        A0[e] = (r < N && c < N && r != c) ? A[(int64_t)r * N + c] : cz();
        if (r == c) d[r] = (r < N) ? A[(int64_t)r * N + r] : make_double2(1.0, 0.0);
    }
}

__global__ void __launch_bounds__(64) fill_u32_kernel(unsigned* __restrict__ p, int count) {
    for (int i = threadIdx.x; i < count; i += 64) p[i] = 0u;
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

// Folds np partial records into one record (sum, compensation, sum|t|) in the
// same layout, with the tree of final_reduce_kernel.
__global__ void __launch_bounds__(256) partials_fold_kernel(const double* __restrict__ partials, int64_t np,
                                                            double* __restrict__ record) {
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
    if (t < 5) record[t] = sh[t][0];
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

// Self-check of the cross-lane sums used above: in[64] -> out[1408]
// (octet sums, stride-8 sums, readlane of lane 37, wave_shr:1, the two swaps,
// six stride-8 sums at once (the 8x8 grid's row sums and the column-swap map's
// column sums), four row sums of the default 8x4 map and four sums over lane
// quads (the column-swap map's row sums)).
__global__ void __launch_bounds__(64) selftest_kernel(const double* __restrict__ in, double* __restrict__ out) {
    const int l = threadIdx.x;
    const double x = in[l];
    out[l] = sum_octet(x);
    out[64 + l] = sum_stride8(x);
    out[128 + l] = readlane_d(x, 37);
    out[192 + l] = dpp_mov<0x138>(x);
    double a = x, b = -x;
    swap16(a, b);
    out[256 + l] = a;
    out[320 + l] = b;
    a = x;
    b = -x;
    swap32(a, b);
    out[384 + l] = a;
    out[448 + l] = b;
    double v[6] = {x, 2.0 * x, 3.0 * x, -x, 0.5 * x, 7.0 * x};
    rowsum_many<8, 8, false, 6>(v);
    for (int j = 0; j < 6; ++j) out[512 + 64 * j + l] = v[j];
    double w[4] = {x, -2.0 * x, 3.0 * x, 0.25 * x};
    rowsum_many<8, 4, false, 4>(w);
    for (int j = 0; j < 4; ++j) out[896 + 64 * j + l] = w[j];
    double u[4] = {x, 0.5 * x, -3.0 * x, 2.0 * x};
    rowsum_many<8, 4, true, 4>(u);
    for (int j = 0; j < 4; ++j) out[1152 + 64 * j + l] = u[j];
}

// ---------------------------------------------------------------- launchers

hipError_t launch_charpoly_l44(const LaunchPhase1& p, hipStream_t st);
hipError_t launch_charpoly_l84(const LaunchPhase1& p, hipStream_t st, bool one_team);
hipError_t launch_charpoly_l88(const LaunchPhase1& p, hipStream_t st);

bool charpoly_layout_ok(int m, int layout) {
    switch (layout) {
        case kLayout44: return m <= 24;
        case kLayout84: return m <= 40;
        case kLayout88: return m <= kMaxTileM;
        case kLayout84T: return m <= 40;
    }
    return false;
}

int charpoly_default_layout(int m) { return m <= 16 ? kLayout44 : (m <= 32 ? kLayout84 : kLayout88); }

hipError_t launch_charpoly_batch_l44(int s_rep, int variant, int offset, int D_max, int fp32, const BatchTile* tiles, int ntiles,
                                     const BatchItem* items, const uint64_t* binom, const int4* lbmap, unsigned* counter, void* Ebase,
                                     int max_grid, hipStream_t st);
hipError_t launch_charpoly_batch_l84(int s_rep, int variant, int offset, int D_max, int fp32, const BatchTile* tiles, int ntiles,
                                     const BatchItem* items, const uint64_t* binom, const int4* lbmap, unsigned* counter, void* Ebase,
                                     int max_grid, hipStream_t st);
hipError_t launch_charpoly_batch_l88(int s_rep, int variant, int offset, int D_max, int fp32, const BatchTile* tiles, int ntiles,
                                     const BatchItem* items, const uint64_t* binom, const int4* lbmap, unsigned* counter, void* Ebase,
                                     int max_grid, hipStream_t st);

int charpoly_instance(int layout, int s) {
    const int m = 2 * s;
    switch (layout) {
        case kLayout44: return 100 + (m + 3) / 4;
        case kLayout84: return 200 + (m + 3) / 4;
        case kLayout84T: return 400 + (m + 3) / 4;
        default: return 300 + (m + 7) / 8;
    }
}

int charpoly_variant(int layout, int n) {
    if (layout == kLayout84T) return 1;
    const int G = (layout == kLayout44) ? 16 : (layout == kLayout84) ? 32 : 64;
    return lb_variant(G, n + 1);
}

// Lane map of a La Budde team of T lanes carrying coefficients 0..D.
// Coefficient d >= 2 has d - 1 terms; it gets g_d = 2^ceil(log2(ceil((d-1)/CH)))
// lanes (capped at 4) with CH the smallest chunk for which all groups fit in
// T lanes, each lane taking a contiguous run of about (d-1)/g_d terms.  Groups
// are laid out from the largest d down, so team lane 0 leads the largest group.
static void lb_fill_one(int T, int D, int4* out) {
    auto p2 = [](int x) { int p = 1; while (p < x) p *= 2; return p; };
    int g[kLbMaxD] = {0};
    bool fit = false;
    for (int ch = 1; ch <= D && !fit; ++ch) {
        int tot = 0;
        bool capped = true;
        for (int d = 0; d <= D; ++d) {
            g[d] = (d < 2) ? 1 : p2((d - 1 + ch - 1) / ch);
            capped = capped && g[d] <= 4;
            tot += g[d];
        }
        fit = capped && tot <= T;
    }
    if (!fit)
        for (int d = 0; d <= D; ++d) g[d] = 1;  // one lane per coefficient (D + 1 <= T)
    for (int l = 0; l < 64; ++l) out[l] = make_int4(-1, 1, 1, 0);
    int start = 0;
    for (int d = D; d >= 0; --d) {
        const int cs = (d >= 2) ? (d - 1 + g[d] - 1) / g[d] : 0;
        for (int c = 0; c < g[d]; ++c) {
            const int klo = 1 + c * cs;
            const int khi = (d >= 2) ? std::min(d - 1, (c + 1) * cs) : 0;
            out[start + c] = make_int4(d, g[d], klo, khi);
        }
        start += g[d];
    }
}

void lb_fill_table(int4* out) {
    const int teams[3] = {16, 32, 64};
    for (int ti = 0; ti < 3; ++ti)
        for (int D = 0; D < kLbMaxD; ++D) {
            int4* o = out + lb_table_offset(teams[ti], D);
            if (D + 1 <= teams[ti]) {
                lb_fill_one(teams[ti], D, o);
            } else {
                for (int l = 0; l < 64; ++l) o[l] = make_int4(-1, 1, 1, 0);
            }
        }
}

hipError_t launch_charpoly_batch(int layout, int s_rep, int variant, int offset, int D_max, int fp32,
                                 const BatchTile* tiles, int ntiles, const BatchItem* items, const uint64_t* binom,
                                 const int4* lbmap, unsigned* counter, void* Ebase, int max_grid, hipStream_t st) {
    if (fp32 && offset != 0) return hipErrorInvalidValue;
    if (!charpoly_layout_ok(2 * s_rep, layout)) return hipErrorInvalidValue;
    if ((layout == kLayout84 || layout == kLayout84T) && 2 * s_rep > kMaxBatchM84) return hipErrorInvalidValue;
    switch (layout) {
        case kLayout44:
            return launch_charpoly_batch_l44(s_rep, variant, offset, D_max, fp32, tiles, ntiles, items, binom, lbmap, counter, Ebase, max_grid, st);
        case kLayout84:
        case kLayout84T:
            return launch_charpoly_batch_l84(s_rep, variant, offset, D_max, fp32, tiles, ntiles, items, binom, lbmap, counter, Ebase, max_grid, st);
        default:
            return launch_charpoly_batch_l88(s_rep, variant, offset, D_max, fp32, tiles, ntiles, items, binom, lbmap, counter, Ebase, max_grid, st);
    }
}

template <int NN>
static hipError_t launch_series_batch_nn(int fp32, const SeriesBlock* blocks, int nblocks, const BatchTile* tiles,
                                         const void* Ebase, int per_thread, double* partials, hipStream_t st) {
    if (fp32)
        hipLaunchKernelGGL((series_batch_kernel<NN, float2>), dim3(nblocks), dim3(64), 0, st, blocks, tiles,
                           static_cast<const float2*>(Ebase), per_thread, partials);
    else
        hipLaunchKernelGGL((series_batch_kernel<NN, double2>), dim3(nblocks), dim3(64), 0, st, blocks, tiles,
                           static_cast<const double2*>(Ebase), per_thread, partials);
    return hipGetLastError();
}

template <int NN>
static hipError_t series_batch_dispatch(int n, int fp32, const SeriesBlock* blocks, int nblocks,
                                        const BatchTile* tiles, const void* Ebase, int per_thread, double* partials,
                                        hipStream_t st) {
    if constexpr (NN > kMaxPairs) {
        return hipErrorInvalidValue;
    } else {
        if (n == NN) return launch_series_batch_nn<NN>(fp32, blocks, nblocks, tiles, Ebase, per_thread, partials, st);
        return series_batch_dispatch<NN + 1>(n, fp32, blocks, nblocks, tiles, Ebase, per_thread, partials, st);
    }
}

hipError_t launch_series_batch(int n, int fp32, const SeriesBlock* blocks, int nblocks, const BatchTile* tiles,
                               const BatchItem* items, const void* Ebase, int per_thread, double* partials,
                               hipStream_t st) {
    (void)items;
    if (nblocks <= 0) return hipSuccess;
    return series_batch_dispatch<1>(n, fp32, blocks, nblocks, tiles, Ebase, per_thread, partials, st);
}

// ---------------------------------------------------------------- small items

namespace {

// Series of one subset for n <= kSmallPairs pairs given at run time: the loops
// are unrolled to kSmallPairs and guarded, so every array index is constant.
__device__ __forceinline__ double2 series_term_small(const double2* __restrict__ E, int n, int RS, double sign) {
    constexpr int NM = kSmallPairs;
    double2 R[NM + 2], c[NM + 1], Lk[NM + 1], p[NM + 1], e[NM + 1];
#pragma unroll
    for (int k = 0; k <= NM + 1; ++k) R[k] = (k <= n + 1) ? E[k] : cz();
    Lk[0] = cz();
    p[0] = cz();
    c[0] = cz();
#pragma unroll
    for (int k = 1; k <= NM; ++k) {
        if (k <= n) {
            const double2 rp = E[RS + k + 1];
            double2 acc = make_double2(R[k + 1].x - rp.x, R[k + 1].y - rp.y);
#pragma unroll
            for (int j = 1; j < k; ++j) acc = cfms(R[j], Lk[k - j], acc);
            Lk[k] = acc;
            double2 pk = make_double2(-(double)k * R[k].x, -(double)k * R[k].y);
#pragma unroll
            for (int j = 1; j < k; ++j) pk = cfms(R[j], p[k - j], pk);
            p[k] = pk;
            const double hk = 0.5 / (double)k;
            c[k] = make_double2(fma(pk.x, hk, 0.5 * acc.x), fma(pk.y, hk, 0.5 * acc.y));
        } else {
            Lk[k] = p[k] = c[k] = cz();
        }
    }
    e[0] = make_double2(1.0, 0.0);
    double2 res = cz();
#pragma unroll
    for (int k = 1; k <= NM; ++k) {
        double2 acc = cz();
#pragma unroll
        for (int j = 1; j <= k; ++j) acc = cfms(make_double2(-(double)j * c[j].x, -(double)j * c[j].y), e[k - j], acc);
        const double ik = 1.0 / (double)k;
        e[k] = make_double2(acc.x * ik, acc.y * ik);
        if (k == n) res = make_double2(e[k].x * sign, e[k].y * sign);
    }
    return res;
}

// One wavefront per loop hafnian with 1 <= n <= kSmallPairs pairs: all its
// subsets in groups of four (4x4 lane grid, the register tile of the subset
// size), each group's series on four lanes, per-lane TwoSum, then a fixed-order
// merge.  Items are taken from `list` (largest first) with a grid stride.
__global__ void __launch_bounds__(64) small_items_kernel(const int* __restrict__ list, int count,
                                                         const BatchItem* __restrict__ items,
                                                         const uint64_t* __restrict__ binom,
                                                         const int4* __restrict__ lbmap, double2* __restrict__ out,
                                                         double* __restrict__ abs_out) {
    extern __shared__ double2 lds[];
    constexpr int W = 4;
    const int lane = threadIdx.x;
    double2* E = lds + charpoly_lds_bytes(W, 16, kSmallPairs + 1, sizeof(double2)) / sizeof(double2);
    for (int w = blockIdx.x; w < count; w += gridDim.x) {
        const int i = __builtin_amdgcn_readfirstlane(list[w]);
        const BatchItem it = items[i];
        const int n = it.n, D = n + 1, RS = D + 1;
        const int4* lbm = lbmap + lb_table_offset(16, D);
        Acc A{0.0, 0.0, 0.0, 0.0, 0.0};
        for (int s = 1; s <= n; ++s) {
            const uint64_t cnt = binom[n * kBinomStride + s];
            const double sign = ((n - s) & 1) ? -1.0 : 1.0;
            const int mr = (2 * s + 3) / 4;
            uint64_t chain = 0;
            for (uint64_t first = 0; first < cnt; first += W) {
                switch (mr) {
                    case 1:
                        charpoly_wave<4, 4, 1, 1, double2, 16, 0, true>(it.A0, it.dvec, it.Np, s, first, cnt - first, 0, nullptr,
                                                               binom, D, lbm, E, lds, chain);
                        break;
                    case 2:
                        charpoly_wave<4, 4, 2, 2, double2, 16, 0, true>(it.A0, it.dvec, it.Np, s, first, cnt - first, 0, nullptr,
                                                               binom, D, lbm, E, lds, chain);
                        break;
                    case 3:
                        charpoly_wave<4, 4, 3, 3, double2, 16, 0, true>(it.A0, it.dvec, it.Np, s, first, cnt - first, 0, nullptr,
                                                               binom, D, lbm, E, lds, chain);
                        break;
                    default:
                        charpoly_wave<4, 4, 4, 4, double2, 16, 0, true>(it.A0, it.dvec, it.Np, s, first, cnt - first, 0, nullptr,
                                                               binom, D, lbm, E, lds, chain);
                        break;
                }
                wave_sync();
                if (lane < W && first + lane < cnt) acc_add(A, series_term_small(E + lane * 2 * RS, n, RS, sign));
                wave_sync();
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
            out[i] = make_double2(A.sr + A.cr, A.si + A.ci);
            if (abs_out) abs_out[i] = A.ab;
        }
    }
}

}  // namespace

hipError_t launch_small_items(const int* list, int count, const BatchItem* items, const uint64_t* binom,
                              const int4* lbmap, double2* out, double* abs_out, int grid, hipStream_t st) {
    if (count <= 0) return hipSuccess;
    static_assert(kSmallPairs + 2 <= 16, "the 16-lane La Budde team must hold D + 1 coefficients");
    const size_t lds = charpoly_lds_bytes(4, 16, kSmallPairs + 1, sizeof(double2)) +
                       sizeof(double2) * 4 * 2 * (kSmallPairs + 2);
    hipLaunchKernelGGL(small_items_kernel, dim3(std::max(1, std::min(grid, count))), dim3(64), lds, st, list, count,
                       items, binom, lbmap, out, abs_out);
    return hipGetLastError();
}

hipError_t launch_item_reduce(const int64_t* pbeg, int nitems, const double* partials, const BatchItem* items,
                              double2* out, double* abs_out, hipStream_t st) {
    if (nitems <= 0) return hipSuccess;
    hipLaunchKernelGGL(item_reduce_kernel, dim3(nitems), dim3(64), 0, st, pbeg, partials, items, out, abs_out);
    return hipGetLastError();
}

hipError_t launch_batch_prep(const double2* mats, const int64_t* in_off, const int* N, BatchItem* items, int nitems,
                             hipStream_t st) {
    if (nitems <= 0) return hipSuccess;
    hipLaunchKernelGGL(batch_prep_kernel, dim3(nitems), dim3(256), 0, st, mats, in_off, N, items);
    return hipGetLastError();
}

hipError_t launch_fill_u32(unsigned* p, int count, hipStream_t st) {
    hipLaunchKernelGGL(fill_u32_kernel, dim3(1), dim3(64), 0, st, p, count);
    return hipGetLastError();
}

hipError_t launch_charpoly(const LaunchPhase1& p, int layout, hipStream_t st) {
    const int m = 2 * p.s;
    if (!charpoly_layout_ok(m, layout)) return hipErrorInvalidValue;
    switch (layout) {
        case kLayout44: return launch_charpoly_l44(p, st);
        case kLayout84: return launch_charpoly_l84(p, st, false);
        case kLayout84T: return launch_charpoly_l84(p, st, true);
        default: return launch_charpoly_l88(p, st);
    }
}

template <int NN>
static hipError_t launch_series_nn(const LaunchPhase2& p, hipStream_t st) {
    const uint64_t per_block = 64ull * p.per_thread;
    const unsigned grid = (unsigned)((p.count + per_block - 1) / per_block);
    if (p.fp32)
        hipLaunchKernelGGL((series_kernel<NN, float2>), dim3(grid), dim3(64), 0, st, static_cast<const float2*>(p.E),
                           p.count, p.D, p.sign, p.per_thread, p.partials, p.terms);
    else
        hipLaunchKernelGGL((series_kernel<NN, double2>), dim3(grid), dim3(64), 0, st,
                           static_cast<const double2*>(p.E), p.count, p.D, p.sign, p.per_thread, p.partials, p.terms);
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

hipError_t launch_partials_fold(const double* partials, int64_t np, double* record, hipStream_t st) {
    hipLaunchKernelGGL(partials_fold_kernel, dim3(1), dim3(256), 0, st, partials, np, record);
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
