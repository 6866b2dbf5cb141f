// Adjoint Gauss-Newton direction for the per-element stiffness gamma_s at the
// equilibrium of one implicit Euler step (Sec. 6.1-6.2: Eq. g, Eq. pxpgamma,
// Eq. adjoint_state, Eq. adjoint_state_solve, Eq. gn, Eq. agn).
//
// With g(x, gamma) = M (x - y) / dt^2 + sum_e G_e^T (w_s (F - R) + w_v (F - V))
// (the equilibrium condition of the step energy whose minimiser the PD
// iteration of Sec. 7.1 converges to), A = dg/dx, B = dg/dgamma_s and the loss
// eps = 1/2 ||x - x_target||^2 over the free vertices (G = I):
//   gradient   grad = -B^T lambda,  A lambda = x - x_target
//   direction  (B^T A^{-1} A^{-1} B + kappa I) d = -grad
// which is Eq. agn's saddle system with its first two block rows eliminated:
// mu = A^{-1} B d, nu = A^{-1} mu.  The direction is found by conjugate
// gradients in gamma space; every product with the GN matrix takes two solves
// with A, by conjugate gradients preconditioned with the decomposed solve of K
// (A = K - sum_e G_e^T J_P G_e, so K^{-1} A is close to the identity while the
// strain is small).  All vectors are FP64; the projection Jacobian and the
// interior solves of the preconditioner run in FP32 as in the step.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <string>
#include <vector>

#include "runtime.h"

using namespace vhrt;

namespace {

struct Buffers {
    vh_ctx* ctx = nullptr;
    std::vector<void*> p;
    size_t bytes = 0;
    ~Buffers() {
        for (void* q : p) (void)hipFree(q);
        if (ctx) uncharge(ctx, bytes);
    }
    int get(double** out, size_t count) {
        const size_t b = std::max<size_t>(count, 1) * sizeof(double);
        if (ctx->budget && ctx->in_use + b > ctx->budget) return fail(VH_ENOMEM, "HBM budget exceeded (Gauss-Newton)");
        void* q = nullptr;
        hipError_t e = hipMalloc(&q, b);
        if (e != hipSuccess) return fail(VH_ENOMEM, std::string("hipMalloc: ") + hipGetErrorString(e));
        p.push_back(q);
        bytes += b;
        charge(ctx, b);
        *out = static_cast<double*>(q);
        return hipMemset(q, 0, b) == hipSuccess ? VH_OK : fail(VH_EDEVICE, "hipMemset");
    }
};

struct GN {
    vh_mesh* m = nullptr;
    hipStream_t s = nullptr;
    const vh::DevMesh* G = nullptr;   // device record of the mesh
    int32_t nt = 0, nf3 = 0;
    size_t nv3 = 0;
    double* x = nullptr;              // equilibrium positions [nv][3], internal order
    double* zero = nullptr;           // [nv][3] zeros
    double* geo = nullptr;            // [nv][3] J_P term of A v
    double* junk_v = nullptr;         // [nv][3] unused outputs of the shared kernels
    double* junk_e = nullptr;         // [nt]
    double* part = nullptr;           // dot-product partials
    std::vector<double> hpart;
    int64_t inner_iters = 0;
    double inner_worst = 0.0;

    int dot(int32_t n, const double* a, const double* b, double* out) {
        VH_HIP(vh::launch_gn_dot(n, a, b, part, s));
        VH_HIP(hipMemcpyAsync(hpart.data(), part, hpart.size() * sizeof(double), hipMemcpyDeviceToHost, s));
        VH_HIP(hipStreamSynchronize(s));
        double acc = 0.0;
        for (double v : hpart) acc += v;
        *out = acc;
        return VH_OK;
    }

    // out = A v (free rows; v's pinned rows are zero)
    int apply_A(const double* v, double* out) {
        VH_HIP(vh::launch_adj_local(G, nt, x, x, v, junk_e, s));
        VH_HIP(vh::launch_adj_gather(G, m->dm.n_free, zero, geo, junk_v, s));
        VH_HIP(vh::launch_gn_av(G, m->dm.n_free, v, geo, out, s));
        return VH_OK;
    }

    // out = K^{-1} r by the decomposed solve of the step
    int precond(const double* r, double* out) {
        VH_HIP(hipMemcpyAsync(m->dm.r, r, (size_t)nf3 * sizeof(double), hipMemcpyDeviceToDevice, s));
        VH_TRY(solve(nullptr, m->ls, s, false, true));
        VH_HIP(hipMemcpyAsync(out, m->dm.delta, (size_t)nf3 * sizeof(double), hipMemcpyDeviceToDevice, s));
        return VH_OK;
    }

    // z = A^{-1} w by preconditioned conjugate gradients (work: r, sv, p, q)
    int solve_A(const double* w, double* z, double* r, double* sv, double* p, double* q, double tol, int32_t max_it) {
        VH_HIP(hipMemsetAsync(z, 0, nv3 * sizeof(double), s));
        VH_HIP(hipMemcpyAsync(r, w, (size_t)nf3 * sizeof(double), hipMemcpyDeviceToDevice, s));
        double ww = 0.0;
        VH_TRY(dot(nf3, w, w, &ww));
        if (ww == 0.0) return VH_OK;
        VH_TRY(precond(r, sv));
        VH_HIP(hipMemcpyAsync(p, sv, (size_t)nf3 * sizeof(double), hipMemcpyDeviceToDevice, s));
        double rs = 0.0, rr = ww;
        VH_TRY(dot(nf3, r, sv, &rs));
        int32_t it = 0;
        for (; it < max_it && rr > tol * tol * ww; ++it) {
            VH_TRY(apply_A(p, q));
            double pq = 0.0;
            VH_TRY(dot(nf3, p, q, &pq));
            if (!(pq > 0.0)) return fail(VH_ENUMERIC, "the equilibrium Hessian is not positive definite");
            const double a = rs / pq;
            VH_HIP(vh::launch_gn_axpy(nf3, a, p, z, s));
            VH_HIP(vh::launch_gn_axpy(nf3, -a, q, r, s));
            VH_TRY(dot(nf3, r, r, &rr));
            VH_TRY(precond(r, sv));
            double rs1 = 0.0;
            VH_TRY(dot(nf3, r, sv, &rs1));
            VH_HIP(vh::launch_gn_xpby(nf3, sv, rs1 / rs, p, s));
            rs = rs1;
        }
        inner_iters += it;
        inner_worst = std::max(inner_worst, std::sqrt(rr / ww));
        return VH_OK;
    }
};

}  // namespace

extern "C" int vh_mesh_gn_direction(vh_mesh* m, const double* x_eq, const double* x_target, double kappa,
                                    int32_t max_outer, double outer_tol, double* grad_gamma_s, double* direction,
                                    vh_gn_stats* stats, void* stream) {
    VH_TRY(check_solo(m));
    if (!x_eq || !x_target || !grad_gamma_s || !direction) return fail(VH_EINVAL, "null argument");
    if (!(kappa >= 0.0) || !std::isfinite(kappa)) return fail(VH_EINVAL, "kappa must be finite and >= 0");
    if (max_outer < 0 || !(outer_tol > 0.0) || !(outer_tol < 1.0)) return fail(VH_EINVAL, "bad iteration controls");
    VH_TRY(set_device(m));
    GN g;
    g.m = m;
    g.s = static_cast<hipStream_t>(stream);
    g.G = m->ls.G;
    vh::DevMesh& d = m->dm;
    const vh::Plan& P = m->plan;
    g.nt = d.nt;
    g.nf3 = d.n_free * 3;
    g.nv3 = (size_t)d.nv * 3;
    const size_t nv3 = g.nv3;
    Buffers b;
    b.ctx = m->ctx;
    double *e = nullptr, *lam = nullptr, *grad = nullptr, *dir = nullptr, *rr = nullptr,
           *pp = nullptr, *qq = nullptr, *w = nullptr, *z1 = nullptr, *z2 = nullptr, *r = nullptr, *sv = nullptr,
           *p = nullptr, *q = nullptr, *xt = nullptr;
    VH_TRY(b.get(&g.x, nv3));
    VH_TRY(b.get(&g.zero, nv3));
    VH_TRY(b.get(&g.geo, nv3));
    VH_TRY(b.get(&g.junk_v, nv3));
    VH_TRY(b.get(&g.junk_e, (size_t)g.nt));
    VH_TRY(b.get(&g.part, (size_t)vh::gn_dot_blocks()));
    VH_TRY(b.get(&e, nv3));
    VH_TRY(b.get(&xt, nv3));
    VH_TRY(b.get(&lam, nv3));
    VH_TRY(b.get(&w, nv3));
    VH_TRY(b.get(&z1, nv3));
    VH_TRY(b.get(&z2, nv3));
    VH_TRY(b.get(&r, nv3));
    VH_TRY(b.get(&sv, nv3));
    VH_TRY(b.get(&p, nv3));
    VH_TRY(b.get(&q, nv3));
    VH_TRY(b.get(&grad, (size_t)g.nt));
    VH_TRY(b.get(&dir, (size_t)g.nt));
    VH_TRY(b.get(&rr, (size_t)g.nt));
    VH_TRY(b.get(&pp, (size_t)g.nt));
    VH_TRY(b.get(&qq, (size_t)g.nt));
    g.hpart.assign((size_t)vh::gn_dot_blocks(), 0.0);
    hipStream_t s = g.s;
    // the positions in the mesh's internal order (the mesh's own state is not
    // touched: the kernels read x_eq from this buffer, the preconditioner
    // solves do not update x)
    VH_TRY(put_user(m, x_eq, g.x, true, s));
    VH_TRY(put_user(m, x_target, xt, true, s));
    // e = x - x_target on the free rows
    VH_HIP(hipMemcpyAsync(e, g.x, (size_t)g.nf3 * sizeof(double), hipMemcpyDeviceToDevice, s));
    VH_HIP(vh::launch_gn_axpy(g.nf3, -1.0, xt, e, s));
    const double inner_tol = 1e-10;
    const int32_t inner_max = 500;
    int rc = VH_OK;
    auto done = [&](int code) {
        (void)hipStreamSynchronize(s);     // the buffers are freed on return
        return code;
    };
    // gradient: lambda = A^{-1} e, grad_e = V_e <G_e lambda, R_e - F_e> = -(B^T lambda)_e
    rc = g.solve_A(e, lam, r, sv, p, q, inner_tol, inner_max);
    if (rc != VH_OK) return done(rc);
    if (hipMemsetAsync(grad, 0, (size_t)g.nt * sizeof(double), s) != hipSuccess ||
        vh::launch_adj_local(g.G, g.nt, g.x, g.x, lam, grad, s) != hipSuccess)
        return done(fail(VH_EDEVICE, "gradient launch"));
    // conjugate gradients on (P + kappa I) d = -grad, d = 0 at the start
    if (hipMemcpyAsync(rr, grad, (size_t)g.nt * sizeof(double), hipMemcpyDeviceToDevice, s) != hipSuccess ||
        vh::launch_gn_xpby(g.nt, g.zero, -1.0, rr, s) != hipSuccess ||
        hipMemcpyAsync(pp, rr, (size_t)g.nt * sizeof(double), hipMemcpyDeviceToDevice, s) != hipSuccess)
        return done(fail(VH_EDEVICE, "Gauss-Newton set-up"));
    double rho = 0.0;
    if ((rc = g.dot(g.nt, rr, rr, &rho)) != VH_OK) return done(rc);
    const double rho0 = rho;
    int32_t it = 0;
    for (; it < max_outer && rho > outer_tol * outer_tol * rho0 && rho0 > 0.0; ++it) {
        // qq = B^T A^{-1} A^{-1} B pp + kappa pp
        if (vh::launch_gn_bd(g.G, g.nt, g.x, pp, s) != hipSuccess ||
            vh::launch_adj_gather(g.G, d.n_free, g.zero, w, g.junk_v, s) != hipSuccess)
            return done(fail(VH_EDEVICE, "B d launch"));
        if ((rc = g.solve_A(w, z1, r, sv, p, q, inner_tol, inner_max)) != VH_OK) return done(rc);
        if ((rc = g.solve_A(z1, z2, r, sv, p, q, inner_tol, inner_max)) != VH_OK) return done(rc);
        if (hipMemsetAsync(qq, 0, (size_t)g.nt * sizeof(double), s) != hipSuccess ||
            vh::launch_adj_local(g.G, g.nt, g.x, g.x, z2, qq, s) != hipSuccess ||
            vh::launch_gn_xpby(g.nt, g.zero, -1.0, qq, s) != hipSuccess ||   // B^T z2 = -(kernel's term)
            vh::launch_gn_axpy(g.nt, kappa, pp, qq, s) != hipSuccess)
            return done(fail(VH_EDEVICE, "GN product launch"));
        double pq = 0.0;
        if ((rc = g.dot(g.nt, pp, qq, &pq)) != VH_OK) return done(rc);
        if (!(pq > 0.0)) return done(fail(VH_ENUMERIC, "the Gauss-Newton matrix is not positive definite"));
        const double a = rho / pq;
        if (vh::launch_gn_axpy(g.nt, a, pp, dir, s) != hipSuccess ||
            vh::launch_gn_axpy(g.nt, -a, qq, rr, s) != hipSuccess)
            return done(fail(VH_EDEVICE, "GN update launch"));
        double rho1 = 0.0;
        if ((rc = g.dot(g.nt, rr, rr, &rho1)) != VH_OK) return done(rc);
        if (vh::launch_gn_xpby(g.nt, rr, rho1 / rho, pp, s) != hipSuccess)
            return done(fail(VH_EDEVICE, "GN update launch"));
        rho = rho1;
    }
    std::vector<double> hg((size_t)g.nt), hd((size_t)g.nt);
    if (hipMemcpyAsync(hg.data(), grad, hg.size() * sizeof(double), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipMemcpyAsync(hd.data(), dir, hd.size() * sizeof(double), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return done(fail(VH_EDEVICE, "Gauss-Newton read-back"));
    for (int32_t k = 0; k < g.nt; ++k) {
        grad_gamma_s[P.elem_perm[k]] = hg[k];
        direction[P.elem_perm[k]] = hd[k];
    }
    if (stats) {
        stats->outer_iters = it;
        stats->inner_iters = g.inner_iters;
        stats->outer_rel_residual = rho0 > 0.0 ? std::sqrt(rho / rho0) : 0.0;
        stats->inner_rel_residual_max = g.inner_worst;
    }
    return done(VH_OK);
}
