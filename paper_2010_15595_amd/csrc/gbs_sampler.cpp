// Conditional sampling chain of a pure Gaussian state (Sec. III of the paper,
// its sampling algorithm), C ABI gbs_sample_pure.
//
// Mode k's photon number is drawn from the probabilities of (s_1, .., s_{k-1}, j),
// j = 0..cutoff, of the pure state of modes 1..k that remains once modes
// k+1..M have been measured by heterodyne detection (outcomes drawn first
// from the Husimi distribution of modes 2..M).  In the complex basis
// (Q = Sigma + I/2, alpha = [a; conj(a)]) the conditional state of A = modes
// 1..k given outcomes beta of B = modes k+1..M is
//   Q_A|B = Q_AA - Sigma_AB Q_BB^-1 Sigma_BA,
//   alpha_A|B = alpha_A + G ([beta; conj(beta)] - alpha_B),  G = Sigma_AB Q_BB^-1,
// the complex-basis form of the Gaussian conditioning of Sec. II.  The
// covariance part does not depend on the outcomes, so it is computed once per
// call on the host for every k (O(M^4) flops, M <= 128), together with the
// affine map from the outcomes to the loop weights of Eq. (12):
//   gamma_k = c_k + F_k [beta_B; conj(beta_B)].
// Everything per sample runs on the GPU in lockstep over a group of samples:
// heterodyne outcomes, loop weights and expanded matrices, the loop hafnians
// (batch kernels through an eager runner, since each step's dimensions depend
// on the previous draws), and the draws.  Only the drawn counts come back to
// the host after every step, to size the next step's batch.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <complex>
#include <cstring>
#include <vector>

#include "gbs_internal.h"

using cplx = std::complex<double>;
using namespace gbs_host;

namespace {

constexpr int kGroup = 8192;                          // samples per lockstep group
constexpr int64_t kRoundBytes = (int64_t)2 << 30;     // coefficient buffer per round
constexpr int64_t kTileSubsets = 256;

// Solves (L L^H) X = Bm in place (L lower, n x n; Bm n x r, row-major).
void chol_solve(const std::vector<cplx>& L, int n, std::vector<cplx>& Bm, int r) {
    for (int c = 0; c < r; ++c) {
        for (int i = 0; i < n; ++i) {
            cplx s = Bm[(size_t)i * r + c];
            for (int t = 0; t < i; ++t) s -= L[(size_t)i * n + t] * Bm[(size_t)t * r + c];
            Bm[(size_t)i * r + c] = s / L[(size_t)i * n + i].real();
        }
        for (int i = n - 1; i >= 0; --i) {
            cplx s = Bm[(size_t)i * r + c];
            for (int t = i + 1; t < n; ++t) s -= std::conj(L[(size_t)t * n + i]) * Bm[(size_t)t * r + c];
            Bm[(size_t)i * r + c] = s / L[(size_t)i * n + i].real();
        }
    }
}

// Host precompute of one call: heterodyne factor and the per-k conditional
// parameters, packed for one upload.
struct ChainParams {
    int M = 0;
    std::vector<double> Lh, mh;         // real Cholesky factor and mean of (Re beta, Im beta), modes 2..M
    std::vector<double2> packed;        // per k: B_k (k x k), c_k (k), F_k (k x 2(M-k))
    std::vector<int64_t> off_B, off_c, off_F;
};

gbs_status chain_params(const gbs_z* Q, const gbs_z* alpha, int M, ChainParams& P) {
    const int n = 2 * M;
    P.M = M;
    auto q = [&](int i, int j) { return cplx(Q[(size_t)i * n + j].re, Q[(size_t)i * n + j].im); };
    auto al = [&](int i) { return cplx(alpha[i].re, alpha[i].im); };
    // heterodyne outcomes of modes 2..M: (Re beta, Im beta) = T [beta; conj(beta)],
    // T = [[I, I], [-iI, iI]] / 2, covariance T Q_BB T^H, mean T alpha_B
    const int h = M - 1, dim = 2 * h;
    if (h > 0) {
        std::vector<int> ib(dim);
        for (int t = 0; t < h; ++t) {
            ib[t] = 1 + t;
            ib[h + t] = M + 1 + t;
        }
        auto T = [&](int a, int c) -> cplx {  // 2h x 2h
            const bool re = a < h;
            const int ai = re ? a : a - h, ci = c < h ? c : c - h;
            if (ai != ci) return 0.0;
            if (re) return 0.5;
            return c < h ? cplx(0.0, -0.5) : cplx(0.0, 0.5);
        };
        std::vector<cplx> R((size_t)dim * dim);
        for (int a = 0; a < dim; ++a)
            for (int b = 0; b < dim; ++b) {
                // only two nonzeros per row of T
                cplx s = 0.0;
                const int ca[2] = {a % h, a % h + h}, cb[2] = {b % h, b % h + h};
                for (int x : ca)
                    for (int y : cb) s += T(a, x) * q(ib[x], ib[y]) * std::conj(T(b, y));
                R[(size_t)a * dim + b] = cplx(s.real(), 0.0);
            }
        if (!cholesky(R, dim)) return fail(GBS_E_NOT_PD, "heterodyne covariance of modes 2..M is not positive definite");
        P.Lh.resize((size_t)dim * dim);
        for (size_t i = 0; i < R.size(); ++i) P.Lh[i] = R[i].real();
        P.mh.resize(dim);
        for (int a = 0; a < dim; ++a) {
            cplx s = 0.0;
            for (int x : {a % h, a % h + h}) s += T(a, x) * al(ib[x]);
            P.mh[a] = s.real();
        }
    }
    // conditional states of modes 1..k given heterodyne outcomes of k+1..M
    P.off_B.resize(M + 1);
    P.off_c.resize(M + 1);
    P.off_F.resize(M + 1);
    int64_t tot = 0;
    for (int k = 1; k <= M; ++k) {
        P.off_B[k] = tot;
        tot += (int64_t)k * k;
        P.off_c[k] = tot;
        tot += k;
        P.off_F[k] = tot;
        tot += (int64_t)k * 2 * (M - k);
    }
    P.packed.assign((size_t)tot, make_double2(0.0, 0.0));
    for (int k = 1; k <= M; ++k) {
        const int na = 2 * k, nb = 2 * (M - k);
        std::vector<int> ia(na), ib(nb);
        for (int i = 0; i < k; ++i) {
            ia[i] = i;
            ia[k + i] = M + i;
        }
        for (int t = 0; t < M - k; ++t) {
            ib[t] = k + t;
            ib[(M - k) + t] = M + k + t;
        }
        // X = Q_BB^-1 Sigma_BA (Sigma_BA = Q_BA: A and B are disjoint), G = X^H
        std::vector<cplx> X((size_t)nb * na), QA((size_t)na * na);
        for (int a = 0; a < na; ++a)
            for (int b = 0; b < na; ++b) QA[(size_t)a * na + b] = q(ia[a], ia[b]);
        if (nb > 0) {
            std::vector<cplx> LB((size_t)nb * nb);
            for (int a = 0; a < nb; ++a)
                for (int b = 0; b < nb; ++b) LB[(size_t)a * nb + b] = q(ib[a], ib[b]);
            if (!cholesky(LB, nb)) return fail(GBS_E_NOT_PD, "Q of modes %d..%d is not positive definite", k + 1, M);
            for (int a = 0; a < nb; ++a)
                for (int b = 0; b < na; ++b) X[(size_t)a * na + b] = q(ib[a], ia[b]);
            chol_solve(LB, nb, X, na);
            // Q_A|B = Q_AA - Sigma_AB X
            for (int a = 0; a < na; ++a)
                for (int b = 0; b < na; ++b) {
                    cplx s = 0.0;
                    for (int t = 0; t < nb; ++t) s += q(ia[a], ib[t]) * X[(size_t)t * na + b];
                    QA[(size_t)a * na + b] -= s;
                }
        }
        // Q_A|B^-1 column by column
        std::vector<cplx> LA(QA);
        if (!cholesky(LA, na)) return fail(GBS_E_NOT_PD, "conditional Q of modes 1..%d is not positive definite", k);
        std::vector<cplx> Qi((size_t)na * na, 0.0);
        for (int i = 0; i < na; ++i) Qi[(size_t)i * na + i] = 1.0;
        chol_solve(LA, na, Qi, na);
        // B_k = (X (I - Q^-1))[:k, :k] = -Q^-1[k + i][j]; the block [:k, k:] vanishes for a pure state
        double qmax = 1.0, off = 0.0;
        for (int i = 0; i < k; ++i)
            for (int j = 0; j < k; ++j) {
                const cplx b = -Qi[(size_t)(k + i) * na + j];
                qmax = std::max(qmax, std::abs(b));
                off = std::max(off, std::abs(Qi[(size_t)(k + i) * na + k + j] - (i == j ? 1.0 : 0.0)));
                P.packed[P.off_B[k] + (size_t)i * k + j] = make_double2(b.real(), b.imag());
            }
        if (off > 1e-8 * qmax)
            return fail(GBS_E_NOT_PURE, "conditional state of modes 1..%d is not pure (off-block %.3g)", k, off);
        // alpha_A|B = (alpha_A - G alpha_B) + G [beta; conj(beta)]; gamma = (Q_A|B^-1 alpha_A|B)[k:]
        std::vector<cplx> a0(na);
        for (int a = 0; a < na; ++a) {
            cplx s = al(ia[a]);
            for (int t = 0; t < nb; ++t) s -= std::conj(X[(size_t)t * na + a]) * al(ib[t]);
            a0[a] = s;
        }
        for (int i = 0; i < k; ++i) {
            cplx s = 0.0;
            for (int a = 0; a < na; ++a) s += Qi[(size_t)(k + i) * na + a] * a0[a];
            P.packed[P.off_c[k] + i] = make_double2(s.real(), s.imag());
            for (int t = 0; t < nb; ++t) {
                cplx f = 0.0;  // (Q^-1 G)[k + i][t], G[a][t] = conj(X[t][a])
                for (int a = 0; a < na; ++a) f += Qi[(size_t)(k + i) * na + a] * std::conj(X[(size_t)t * na + a]);
                P.packed[P.off_F[k] + (size_t)i * nb + t] = make_double2(f.real(), f.imag());
            }
        }
    }
    return GBS_OK;
}

// Device buffers of one call.
struct ChainDev {
    double *L = nullptr, *mean = nullptr, *normals = nullptr, *uniforms = nullptr, *probs = nullptr;
    double2 *params = nullptr, *beta = nullptr;
    int* draws = nullptr;
    ~ChainDev() {
        void* b[] = {L, mean, normals, uniforms, probs, params, beta, draws};
        for (void* p : b)
            if (p) (void)hipFree(p);
    }
};

template <class T>
gbs_status dalloc(T** p, size_t n) {
    const hipError_t e = dev_malloc((void**)p, std::max<size_t>(1, n) * sizeof(T));
    if (e != hipSuccess) {
        *p = nullptr;
        return fail(GBS_E_NOMEM, "hipMalloc(%zu) failed: %s", n * sizeof(T), hipGetErrorString(e));
    }
    return GBS_OK;
}

}  // namespace

extern "C" gbs_status gbs_sample_pure(const gbs_z* Q, const gbs_z* alpha, int32_t M, int32_t cutoff,
                                      const double* normals, const double* uniforms, int32_t nsamples,
                                      gbs_precision prec, int32_t* samples_out, double* probs_out,
                                      gbs_sample_info* info) {
    const auto t_start = std::chrono::steady_clock::now();
    if (M < 1 || cutoff < 0 || nsamples < 0) return fail(GBS_E_ARG, "bad sizes (M %d, cutoff %d, samples %d)", M, cutoff,
                                                         nsamples);
    if (!Q || !alpha) return fail(GBS_E_ARG, "null Q or alpha");
    if (nsamples > 0 && (!uniforms || !samples_out || (M > 1 && !normals)))
        return fail(GBS_E_ARG, "null random inputs or output");
    if (prec == GBS_DD) return fail(GBS_E_UNSUPPORTED, "the sampling chain runs in FP64 or FP32_COMP");
    if (prec != GBS_FP64 && prec != GBS_FP32_COMP) return fail(GBS_E_ARG, "bad precision %d", (int)prec);
    if (M > gbs::kMaxSamplerModes) return fail(GBS_E_TOO_LARGE, "%d modes exceed %d", M, gbs::kMaxSamplerModes);
    if (cutoff > gbs::kMaxTileM) return fail(GBS_E_TOO_LARGE, "cutoff %d exceeds %d", cutoff, gbs::kMaxTileM);
    for (int64_t i = 0; i < (int64_t)nsamples * 2 * (M - 1); ++i)
        if (!std::isfinite(normals[i])) return fail(GBS_E_NONFINITE, "non-finite normal %lld", (long long)i);
    for (int64_t i = 0; i < (int64_t)nsamples * M; ++i)
        if (!(uniforms[i] >= 0.0 && uniforms[i] < 1.0))
            return fail(GBS_E_ARG, "uniform %lld = %g is not in [0, 1)", (long long)i, uniforms[i]);
    // validates Q and alpha (finite, Hermitian positive definite, pure)
    gbs_status st = gbs_pure_state(Q, alpha, M, nullptr, nullptr, nullptr);
    if (st != GBS_OK) return st;
    ChainParams P;
    st = chain_params(Q, alpha, M, P);
    if (st != GBS_OK) return st;
    const double setup_ms =
        std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_start).count();

    std::lock_guard<std::mutex> lock(g_mutex);
    DevCtx* c = nullptr;
    st = current_ctx(&c);
    if (st != GBS_OK) return st;
    if (!c->runner && (st = runner_create(c, &c->runner)) != GBS_OK) return st;
    hipStream_t s = c->stream;
    HIP_TRY(hipStreamWaitEvent(s, c->done, 0));
    const int group = std::min(std::max(nsamples, 1), kGroup);
    const int h = M - 1, dim = 2 * h, K1 = cutoff + 1;
    ChainDev d;
    if ((st = dalloc(&d.L, P.Lh.size())) != GBS_OK || (st = dalloc(&d.mean, P.mh.size())) != GBS_OK ||
        (st = dalloc(&d.params, P.packed.size())) != GBS_OK || (st = dalloc(&d.normals, (size_t)group * dim)) != GBS_OK ||
        (st = dalloc(&d.uniforms, (size_t)group * M)) != GBS_OK || (st = dalloc(&d.beta, (size_t)group * h)) != GBS_OK ||
        (st = dalloc(&d.draws, (size_t)group * M)) != GBS_OK)
        return st;
    if (probs_out && (st = dalloc(&d.probs, (size_t)group * M * K1)) != GBS_OK) return st;
    if (!P.Lh.empty()) HIP_TRY(hipMemcpy(d.L, P.Lh.data(), P.Lh.size() * sizeof(double), hipMemcpyHostToDevice));
    if (!P.mh.empty()) HIP_TRY(hipMemcpy(d.mean, P.mh.data(), P.mh.size() * sizeof(double), hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(d.params, P.packed.data(), P.packed.size() * sizeof(double2), hipMemcpyHostToDevice));

    const bool fp32 = prec == GBS_FP32_COMP;
    int64_t n_lhaf = 0, n_terms = 0;
    int max_dim = 0, groups = 0;
    std::vector<double> ut((size_t)group * M);
    std::vector<int> P_tot(group), col(group), dims;
    std::vector<int> all_draws((size_t)group * M);
    for (int g0 = 0; g0 < nsamples; g0 += group) {
        const int G = std::min(group, nsamples - g0);
        ++groups;
        // uniforms mode-major, so that step k reads one contiguous row
        for (int b = 0; b < G; ++b)
            for (int i = 0; i < M; ++i) ut[(size_t)i * G + b] = uniforms[(size_t)(g0 + b) * M + i];
        HIP_TRY(hipMemcpyAsync(d.uniforms, ut.data(), sizeof(double) * (size_t)G * M, hipMemcpyHostToDevice, s));
        if (h > 0) {
            HIP_TRY(hipMemcpyAsync(d.normals, normals + (size_t)g0 * dim, sizeof(double) * (size_t)G * dim,
                                   hipMemcpyHostToDevice, s));
            HIP_TRY(gbs::launch_heterodyne(d.L, d.mean, dim, d.normals, G, d.beta, s));
        }
        std::fill(P_tot.begin(), P_tot.begin() + G, 0);
        for (int k = 1; k <= M; ++k) {
            dims.resize((size_t)G * K1);
            for (int b = 0; b < G; ++b) {
                if (P_tot[b] + cutoff > gbs::kMaxTileM) {
                    HIP_TRY(hipStreamSynchronize(s));
                    return fail(GBS_E_TOO_LARGE,
                                "sample %d holds %d photons before mode %d: its loop hafnians up to cutoff %d "
                                "exceed dimension %d",
                                g0 + b, P_tot[b], k, cutoff, gbs::kMaxTileM);
                }
                for (int j = 0; j < K1; ++j) dims[(size_t)b * K1 + j] = P_tot[b] + j;
            }
            for (int n = 1; n <= (*std::max_element(dims.begin(), dims.end()) + 1) / 2; ++n)
                if ((st = maybe_tune(c, n)) != GBS_OK) return st;
            BatchSchedule S;
            batch_schedule(c, dims, fp32, kTileSubsets, kRoundBytes, false, S);
            n_lhaf += S.count;
            n_terms += S.subset_terms;
            for (int N : dims) max_dim = std::max(max_dim, N);
            if ((st = ensure_buffer(&c->smats, &c->smats_cap, sizeof(double2) * std::max<int64_t>(1, S.in_elems), 1)) !=
                GBS_OK)
                return st;
            gbs::SamplerStep sp{};
            sp.M = M;
            sp.k = k;
            sp.cutoff = cutoff;
            sp.nsamples = G;
            sp.Bk = d.params + P.off_B[k];
            sp.ck = d.params + P.off_c[k];
            sp.Fk = d.params + P.off_F[k];
            sp.beta = d.beta;
            sp.samples = d.draws;
            sp.mats = static_cast<double2*>(c->smats);
            st = runner_run(c->runner, S, sp.mats, s, [&](const int64_t* in_off, const int* dv) -> gbs_status {
                sp.in_off = in_off;
                sp.dims = dv;
                HIP_TRY(gbs::launch_sampler_build(sp, s));
                return GBS_OK;
            });
            if (st != GBS_OK) return st;
            int* draw_k = d.draws + (size_t)(k - 1) * G;
            HIP_TRY(gbs::launch_sampler_draw(runner_out(c->runner), G, cutoff, d.uniforms + (size_t)(k - 1) * G, draw_k,
                                             d.probs ? d.probs + (size_t)(k - 1) * K1 : nullptr, (int64_t)M * K1, s));
            HIP_TRY(hipMemcpyAsync(col.data(), draw_k, sizeof(int) * G, hipMemcpyDeviceToHost, s));
            HIP_TRY(hipStreamSynchronize(s));
            for (int b = 0; b < G; ++b) {
                if (col[b] < 0)
                    return fail(GBS_E_NONFINITE, "conditional probabilities of sample %d at mode %d are not finite or "
                                                 "all zero", g0 + b, k);
                P_tot[b] += col[b];
                all_draws[(size_t)(k - 1) * G + b] = col[b];
            }
        }
        for (int b = 0; b < G; ++b)
            for (int i = 0; i < M; ++i) samples_out[(size_t)(g0 + b) * M + i] = all_draws[(size_t)i * G + b];
        if (probs_out)
            HIP_TRY(hipMemcpy(probs_out + (size_t)g0 * M * K1, d.probs, sizeof(double) * (size_t)G * M * K1,
                              hipMemcpyDeviceToHost));
    }
    HIP_TRY(hipEventRecord(c->done, s));
    HIP_TRY(hipStreamSynchronize(s));
    if (info) {
        info->loop_hafnians = n_lhaf;
        info->subset_terms = n_terms;
        info->max_dim = max_dim;
        info->groups = groups;
        info->setup_ms = setup_ms;
        info->total_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_start).count();
    }
    return GBS_OK;
}
