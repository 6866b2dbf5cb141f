// Host construction of the inexact component-mode-synthesis (CMS) solve of
// Sec. 7.2: per subdomain d the boundary modes Psi_d = -(K_d^ii)^{-1} K_d^ib of
// Eq. cms_boundary (columns: the interface rows adjacent to d's interior) and
// the `modes` eigenvectors Phi_d of K_d^ii with the smallest eigenvalues, and
// the Jacobi polishing data (inverse diagonal of K, the Chebyshev weights of
// the semi-iterative method for the spectral radius rho of I - D^{-1} K).
//
// Numerics (FP64): dense Cholesky of K_d^ii; Psi_d by its triangular solves;
// Phi_d by Lanczos on (K_d^ii)^{-1} with full reorthogonalisation, Ritz pairs
// of the tridiagonal matrix by cyclic Jacobi rotations, the Krylov space grown
// until every kept Ritz pair has residual |K phi - lambda phi| <= 1e-10
// lambda_max (at most the whole interior); rho from the extreme Ritz values
// of a Lanczos run on D^{-1/2} K D^{-1/2}.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <string>
#include <vector>

#include "plan.h"

namespace vh {
namespace {

// A = L L^T in place (lower triangle, row-major n x n); false if not SPD
bool cholesky(std::vector<double>& A, int n) {
    for (int j = 0; j < n; ++j) {
        double* rj = &A[(size_t)j * n];
        double s = rj[j];
        for (int k = 0; k < j; ++k) s -= rj[k] * rj[k];
        if (!(s > 0.0) || !std::isfinite(s)) return false;
        const double d = std::sqrt(s);
        rj[j] = d;
        for (int i = j + 1; i < n; ++i) {
            double* ri = &A[(size_t)i * n];
            double t = ri[j];
            for (int k = 0; k < j; ++k) t -= ri[k] * rj[k];
            ri[j] = t / d;
        }
    }
    return true;
}

// x <- (L L^T)^{-1} x
void chol_solve(const std::vector<double>& L, int n, double* x) {
    for (int i = 0; i < n; ++i) {
        const double* ri = &L[(size_t)i * n];
        double t = x[i];
        for (int k = 0; k < i; ++k) t -= ri[k] * x[k];
        x[i] = t / ri[i];
    }
    for (int i = n - 1; i >= 0; --i) {
        double t = x[i];
        for (int k = i + 1; k < n; ++k) t -= L[(size_t)k * n + i] * x[k];
        x[i] = t / L[(size_t)i * n + i];
    }
}

// Eigen-decomposition of a symmetric m x m matrix (row-major, destroyed) by
// cyclic Jacobi rotations: eigenvalues in w, eigenvectors in the columns of V.
void jacobi_eigen(std::vector<double>& A, int m, std::vector<double>& w, std::vector<double>& V) {
    V.assign((size_t)m * m, 0.0);
    for (int i = 0; i < m; ++i) V[(size_t)i * m + i] = 1.0;
    double fro = 0.0;
    for (double a : A) fro += a * a;
    for (int sweep = 0; sweep < 100; ++sweep) {
        double off = 0.0;
        for (int p = 0; p < m; ++p)
            for (int q = p + 1; q < m; ++q) off += A[(size_t)p * m + q] * A[(size_t)p * m + q];
        if (off <= 1e-32 * fro) break;
        for (int p = 0; p < m; ++p)
            for (int q = p + 1; q < m; ++q) {
                const double apq = A[(size_t)p * m + q];
                if (apq == 0.0) continue;
                const double app = A[(size_t)p * m + p], aqq = A[(size_t)q * m + q];
                const double th = (aqq - app) / (2.0 * apq);
                const double t = (th >= 0 ? 1.0 : -1.0) / (std::fabs(th) + std::sqrt(th * th + 1.0));
                const double c = 1.0 / std::sqrt(t * t + 1.0), s = t * c;
                for (int k = 0; k < m; ++k) {                 // columns p, q
                    const double akp = A[(size_t)k * m + p], akq = A[(size_t)k * m + q];
                    A[(size_t)k * m + p] = c * akp - s * akq;
                    A[(size_t)k * m + q] = s * akp + c * akq;
                }
                for (int k = 0; k < m; ++k) {                 // rows p, q
                    const double apk = A[(size_t)p * m + k], aqk = A[(size_t)q * m + k];
                    A[(size_t)p * m + k] = c * apk - s * aqk;
                    A[(size_t)q * m + k] = s * apk + c * aqk;
                }
                for (int k = 0; k < m; ++k) {
                    const double vkp = V[(size_t)k * m + p], vkq = V[(size_t)k * m + q];
                    V[(size_t)k * m + p] = c * vkp - s * vkq;
                    V[(size_t)k * m + q] = s * vkp + c * vkq;
                }
            }
    }
    w.resize(m);
    for (int i = 0; i < m; ++i) w[i] = A[(size_t)i * m + i];
}

// deterministic start vectors: a fixed linear congruential sequence
void fill_start(std::vector<double>& v, uint64_t seed) {
    uint64_t s = 0x9E3779B97F4A7C15ull ^ seed;
    for (double& x : v) {
        s = s * 6364136223846793005ull + 1442695040888963407ull;
        x = (double)(s >> 11) * (1.0 / 9007199254740992.0) - 0.5;
    }
}

double dot(const double* a, const double* b, int n) {
    double s = 0.0;
    for (int i = 0; i < n; ++i) s += a[i] * b[i];
    return s;
}

// Lanczos on the symmetric operator op (n x n), at most m steps (m <= n): the
// orthonormal basis Q (column-major) and the tridiagonal entries alpha, beta;
// with `reorth` every new vector is orthogonalised against the whole basis
// (twice), without it only the three-term recurrence runs (enough for the
// extreme eigenvalues).  Stops early at an invariant subspace.  Returns the
// number of steps taken.
template <class Op>
int lanczos(Op op, int n, int m, uint64_t seed, bool reorth, std::vector<double>& Q, std::vector<double>& alpha,
            std::vector<double>& beta) {
    Q.assign((size_t)n * m, 0.0);
    alpha.assign(m, 0.0);
    beta.assign(m, 0.0);
    std::vector<double> w(n);
    fill_start(w, seed);
    const double nw = std::sqrt(dot(w.data(), w.data(), n));
    for (int i = 0; i < n; ++i) Q[i] = w[i] / nw;
    int steps = 0;
    for (int j = 0; j < m; ++j) {
        const double* qj = &Q[(size_t)j * n];
        op(qj, w.data());
        alpha[j] = dot(qj, w.data(), n);
        steps = j + 1;
        if (reorth) {
            for (int pass = 0; pass < 2; ++pass)
                for (int i = 0; i <= j; ++i) {
                    const double* qi = &Q[(size_t)i * n];
                    const double c = dot(qi, w.data(), n);
                    for (int k = 0; k < n; ++k) w[k] -= c * qi[k];
                }
        } else {
            for (int k = 0; k < n; ++k) w[k] -= alpha[j] * qj[k];
            if (j > 0) {
                const double* qp = &Q[(size_t)(j - 1) * n];
                for (int k = 0; k < n; ++k) w[k] -= beta[j - 1] * qp[k];
            }
        }
        if (j + 1 == m) break;
        const double b = std::sqrt(dot(w.data(), w.data(), n));
        if (!(b > 1e-13 * std::fabs(alpha[j]))) break;
        beta[j] = b;
        double* qn = &Q[(size_t)(j + 1) * n];
        for (int k = 0; k < n; ++k) qn[k] = w[k] / b;
    }
    return steps;
}

// the `r` smallest eigenpairs of the dense SPD matrix K (row-major n x n) with
// Cholesky factor L: lambda[r], phi[r][n]; false if they do not converge
bool lowest_modes(const std::vector<double>& K, const std::vector<double>& L, int n, int r, uint64_t seed,
                  std::vector<double>& lambda, std::vector<double>& phi) {
    double kmax = 0.0;
    for (int i = 0; i < n; ++i) kmax = std::max(kmax, std::fabs(K[(size_t)i * n + i]));
    auto inv = [&](const double* x, double* y) {
        for (int i = 0; i < n; ++i) y[i] = x[i];
        chol_solve(L, n, y);
    };
    std::vector<double> Q, a, b, T, w, V, Kx(n);
    for (int m = std::min(n, 3 * r + 30);; m = std::min(n, 2 * m)) {
        const int mm = lanczos(inv, n, m, seed, true, Q, a, b);
        T.assign((size_t)mm * mm, 0.0);
        for (int i = 0; i < mm; ++i) {
            T[(size_t)i * mm + i] = a[i];
            if (i + 1 < mm) T[(size_t)i * mm + i + 1] = T[(size_t)(i + 1) * mm + i] = b[i];
        }
        jacobi_eigen(T, mm, w, V);
        std::vector<int> order(mm);
        for (int i = 0; i < mm; ++i) order[i] = i;
        std::sort(order.begin(), order.end(), [&](int x, int y) { return w[x] > w[y]; });   // largest of K^{-1}
        const int rr = std::min(r, mm);
        lambda.assign(r, 0.0);
        phi.assign((size_t)r * n, 0.0);
        bool ok = rr == r;
        for (int k = 0; k < rr; ++k) {
            const int c = order[k];
            double* p = &phi[(size_t)k * n];
            for (int j = 0; j < mm; ++j) {
                const double y = V[(size_t)j * mm + c];
                const double* qj = &Q[(size_t)j * n];
                for (int i = 0; i < n; ++i) p[i] += y * qj[i];
            }
            const double nrm = std::sqrt(dot(p, p, n));
            for (int i = 0; i < n; ++i) p[i] /= nrm;
            lambda[k] = 1.0 / w[c];
            for (int i = 0; i < n; ++i) Kx[i] = dot(&K[(size_t)i * n], p, n) - lambda[k] * p[i];
            if (std::sqrt(dot(Kx.data(), Kx.data(), n)) > 1e-10 * kmax) ok = false;
        }
        if (ok) return true;
        if (m == n) return false;
    }
}

}  // namespace

int build_cms(const Plan& P, int32_t modes, int32_t sweeps, CmsPlan& C, std::string& msg) {
    C = CmsPlan();
    C.modes = modes;
    C.sweeps = sweeps;
    const int32_t D = P.D, nf = P.n_free;
    C.phi_off.assign(D + 1, 0);
    C.psi_off.assign(D + 1, 0);
    for (int32_t d = 0; d < D; ++d) {
        const int64_t ni = P.sub_off[d + 1] - P.sub_off[d], nb = P.bnd_off[d + 1] - P.bnd_off[d];
        C.phi_off[d + 1] = C.phi_off[d] + ni * modes;
        C.psi_off[d + 1] = C.psi_off[d] + ni * nb;
    }
    C.phi.assign((size_t)C.phi_off[D], 0.0f);
    C.psi.assign((size_t)C.psi_off[D], 0.0f);
    C.ilam.assign((size_t)D * modes, 0.0f);
    C.lambda.assign((size_t)D * modes, 0.0);
    std::vector<int> bad(D, 0);
#pragma omp parallel for schedule(dynamic, 1)
    for (int32_t d = 0; d < D; ++d) {
        const int32_t r0 = P.sub_off[d], n = P.sub_off[d + 1] - r0;
        const int32_t b0 = P.bnd_off[d], nb = P.bnd_off[d + 1] - b0;
        if (n == 0) continue;
        std::vector<int32_t> bpos(nf, -1);
        for (int32_t k = 0; k < nb; ++k) bpos[P.bnd[b0 + k]] = k;
        std::vector<double> K((size_t)n * n, 0.0), Kib((size_t)n * std::max(nb, 1), 0.0);
        for (int32_t i = 0; i < n; ++i)
            for (int32_t k = P.K_ptr[r0 + i]; k < P.K_ptr[r0 + i + 1]; ++k) {
                const int32_t c = P.K_col[k];
                if (c >= r0 && c < r0 + n) K[(size_t)i * n + (c - r0)] = P.K_val[k];
                else if (bpos[c] >= 0) Kib[(size_t)i * nb + bpos[c]] = P.K_val[k];
            }
        std::vector<double> L = K;
        if (!cholesky(L, n)) {
            bad[d] = 1;
            continue;
        }
        // Psi_d, column-major: Psi[j][i] = -(K^ii)^{-1} K^ib[:, j]
        std::vector<double> col(n);
        for (int32_t j = 0; j < nb; ++j) {
            for (int32_t i = 0; i < n; ++i) col[i] = -Kib[(size_t)i * nb + j];
            chol_solve(L, n, col.data());
            for (int32_t i = 0; i < n; ++i) C.psi[(size_t)C.psi_off[d] + (size_t)j * n + i] = (float)col[i];
        }
        std::vector<double> lam, phi;
        const int32_t r = std::min(modes, n);
        if (r > 0 && !lowest_modes(K, L, n, r, 1000 + (uint64_t)d, lam, phi)) {
            bad[d] = 2;
            continue;
        }
        for (int32_t k = 0; k < r; ++k) {
            C.lambda[(size_t)d * modes + k] = lam[k];
            C.ilam[(size_t)d * modes + k] = (float)(1.0 / lam[k]);
            for (int32_t i = 0; i < n; ++i)
                C.phi[(size_t)C.phi_off[d] + (size_t)k * n + i] = (float)phi[(size_t)k * n + i];
        }
    }
    for (int32_t d = 0; d < D; ++d) {
        if (bad[d] == 1) {
            msg = "non-positive pivot in a dense interior block (CMS)";
            return -3;
        }
        if (bad[d] == 2) {
            msg = "the interior eigenmodes did not converge (CMS)";
            return -5;
        }
    }
    // Jacobi polishing: D^{-1} and rho(I - D^{-1} K) from the extreme Ritz
    // values of D^{-1/2} K D^{-1/2}
    C.inv_diag.assign(nf, 0.0);
    std::vector<double> ds(nf);
    for (int32_t i = 0; i < nf; ++i) {
        double dv = 0.0;
        for (int32_t k = P.K_ptr[i]; k < P.K_ptr[i + 1]; ++k)
            if (P.K_col[k] == i) dv = P.K_val[k];
        if (!(dv > 0.0)) {
            msg = "non-positive diagonal entry (CMS)";
            return -3;
        }
        C.inv_diag[i] = 1.0 / dv;
        ds[i] = 1.0 / std::sqrt(dv);
    }
    if (sweeps > 0 && nf > 0) {
        auto op = [&](const double* x, double* y) {
            for (int32_t i = 0; i < nf; ++i) {
                double s = 0.0;
                for (int32_t k = P.K_ptr[i]; k < P.K_ptr[i + 1]; ++k) s += P.K_val[k] * ds[P.K_col[k]] * x[P.K_col[k]];
                y[i] = ds[i] * s;
            }
        };
        std::vector<double> Q, a, b, T, w, V;
        const int m = lanczos(op, nf, std::min(nf, 300), 7, false, Q, a, b);
        T.assign((size_t)m * m, 0.0);
        for (int i = 0; i < m; ++i) {
            T[(size_t)i * m + i] = a[i];
            if (i + 1 < m) T[(size_t)i * m + i + 1] = T[(size_t)(i + 1) * m + i] = b[i];
        }
        jacobi_eigen(T, m, w, V);
        const double lo = *std::min_element(w.begin(), w.end()), hi = *std::max_element(w.begin(), w.end());
        C.rho = std::max(std::fabs(1.0 - lo), std::fabs(1.0 - hi));
        for (int32_t k = 0; k < sweeps; ++k) {
            double om = 1.0;
            if (k == 1) om = 2.0 / (2.0 - C.rho * C.rho);
            else if (k > 1) om = 4.0 / (4.0 - C.rho * C.rho * C.omega.back());
            C.omega.push_back(om);
        }
    }
    return 0;
}

}  // namespace vh
