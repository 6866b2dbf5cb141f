// Discrete adjoint of a PD trajectory with respect to the per-element stiffness
// gamma_s: a forward run that keeps (x, v) checkpoints on the device, and a
// reverse sweep that replays each checkpoint segment (keeping every iterate)
// and reverses its frames iteration by iteration.
//
// Per iteration x^(k+1) = L^{-1} b(x^(k)), with lambda = L^{-1} xbar^(k+1) from
// the same decomposed solve as the forward step (L is symmetric):
//   gbar_e  += V_e <G_e lambda, R_e(x^(k)) - F_e(x^(k+1))>
//   xbar^(k) = sum_e G_e^T J_P(F_e(x^(k))) [G_e lambda],   ybar += M lambda / dt^2
// and per frame x^(0) = y = x_n + dt v_n + dt^2 g, v_{n+1} = (x_{n+1} - x_n) / dt.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <string>
#include <vector>

#include "runtime.h"

namespace vhrt {

void free_adjoint(vh_mesh* m) {
    if (m->adj_ckpt) {
        (void)hipFree(m->adj_ckpt);
        if (m->ctx) uncharge(m->ctx, m->adj_ckpt_bytes);
    }
    m->adj_ckpt = nullptr;
    m->adj_ckpt_bytes = 0;
    m->adj_frames = 0;
    m->adj_every = 0;
}

namespace {

// device scratch of one reverse sweep, charged to the context while it lives
struct Scratch {
    vh_ctx* ctx = nullptr;
    std::vector<void*> p;
    size_t bytes = 0;
    ~Scratch() {
        for (void* q : p) (void)hipFree(q);
        if (ctx) uncharge(ctx, bytes);
    }
    int get(double** out, size_t count) {
        const size_t b = std::max<size_t>(count, 1) * sizeof(double);
        if (ctx->budget && ctx->in_use + b > ctx->budget) return fail(VH_ENOMEM, "HBM budget exceeded (adjoint)");
        void* q = nullptr;
        hipError_t e = hipMalloc(&q, b);
        if (e != hipSuccess) return fail(VH_ENOMEM, std::string("hipMalloc: ") + hipGetErrorString(e));
        p.push_back(q);
        bytes += b;
        charge(ctx, b);
        *out = static_cast<double*>(q);
        return VH_OK;
    }
};

int one_frame(vh_mesh* m, hipStream_t s) {
    if (m->ctx->cfg.use_graphs) {
        VH_TRY(ensure_graph(m));
        VH_HIP(hipGraphLaunch(m->gexec, s));
        return VH_OK;
    }
    return frame_direct(nullptr, m->ls, s);
}

}  // namespace
}  // namespace vhrt

using namespace vhrt;

extern "C" {

int vh_mesh_adjoint_forward(vh_mesh* m, const double* x0, const double* v0, int32_t n_frames, int32_t ckpt_every,
                            double* x_final, void* stream) {
    VH_TRY(check_solo(m));
    if (!x0 || !v0 || !x_final) return fail(VH_EINVAL, "null argument");
    if (n_frames < 1 || ckpt_every < 1) return fail(VH_EINVAL, "n_frames and ckpt_every must be >= 1");
    if (m->cms.modes > 0) return fail(VH_EINVAL, "the adjoint reverses the exact global solve, not the CMS solve");
    VH_TRY(set_device(m));
    hipStream_t s = static_cast<hipStream_t>(stream);
    vh::DevMesh& d = m->dm;
    const size_t nv3 = (size_t)d.nv * 3;
    free_adjoint(m);
    const int32_t nck = (n_frames + ckpt_every - 1) / ckpt_every;
    const size_t bytes = (size_t)nck * 2 * nv3 * sizeof(double);
    if (m->ctx->budget && m->ctx->in_use + bytes > m->ctx->budget)
        return fail(VH_ENOMEM, "HBM budget exceeded (adjoint checkpoints)");
    VH_HIP(hipMalloc(reinterpret_cast<void**>(&m->adj_ckpt), bytes));
    m->adj_ckpt_bytes = bytes;
    charge(m->ctx, bytes);
    VH_TRY(put_user(m, x0, d.x, true, s));
    VH_TRY(put_user(m, v0, d.v, false, s));
    VH_HIP(vh::launch_refresh_u(d, s));
    for (int32_t f = 0; f < n_frames; ++f) {
        if (f % ckpt_every == 0) {
            double* ck = m->adj_ckpt + (size_t)(f / ckpt_every) * 2 * nv3;
            VH_HIP(hipMemcpyAsync(ck, d.x, nv3 * sizeof(double), hipMemcpyDeviceToDevice, s));
            VH_HIP(hipMemcpyAsync(ck + nv3, d.v, nv3 * sizeof(double), hipMemcpyDeviceToDevice, s));
        }
        VH_TRY(one_frame(m, s));
    }
    VH_TRY(get_user(m, d.x, x_final, m->plan.nv, s));
    m->adj_frames = n_frames;
    m->adj_every = ckpt_every;
    return VH_OK;
}

int vh_mesh_adjoint_backward(vh_mesh* m, const double* xbar_final, const double* vbar_final, double* grad_gamma_s,
                             void* stream) {
    VH_TRY(check_solo(m));
    if (!xbar_final || !grad_gamma_s) return fail(VH_EINVAL, "null argument");
    if (m->adj_frames < 1 || !m->adj_ckpt) return fail(VH_ESTATE, "vh_mesh_adjoint_forward must come first");
    VH_TRY(set_device(m));
    hipStream_t s = static_cast<hipStream_t>(stream);
    vh::DevMesh& d = m->dm;
    const vh::Plan& P = m->plan;
    const int32_t K = P.pd_iters, every = m->adj_every, n = m->adj_frames;
    const size_t nv3 = (size_t)d.nv * 3;
    const int32_t nf3 = d.n_free * 3;
    const vh::DevMesh* G = m->ls.G;   // device copy of d
    Scratch sc;
    sc.ctx = m->ctx;
    double *it = nullptr, *xbar = nullptr, *vbar = nullptr, *xk = nullptr, *xn = nullptr, *ybar = nullptr,
           *lam = nullptr, *gbar = nullptr;
    VH_TRY(sc.get(&it, (size_t)every * (K + 1) * nv3));
    VH_TRY(sc.get(&xbar, nv3));
    VH_TRY(sc.get(&vbar, nv3));
    VH_TRY(sc.get(&xk, nv3));
    VH_TRY(sc.get(&xn, nv3));
    VH_TRY(sc.get(&ybar, nv3));
    VH_TRY(sc.get(&lam, nv3));
    VH_TRY(sc.get(&gbar, (size_t)d.nt));
    VH_TRY(put_user(m, xbar_final, xbar, false, s));
    if (vbar_final) VH_TRY(put_user(m, vbar_final, vbar, false, s));
    else VH_HIP(hipMemsetAsync(vbar, 0, nv3 * sizeof(double), s));
    VH_HIP(hipMemsetAsync(lam, 0, nv3 * sizeof(double), s));
    VH_HIP(hipMemsetAsync(gbar, 0, (size_t)d.nt * sizeof(double), s));
    const int32_t nck = (n + every - 1) / every;
    for (int32_t seg = nck - 1; seg >= 0; --seg) {
        const int32_t f0 = seg * every, f1 = std::min(n, f0 + every);
        const double* ck = m->adj_ckpt + (size_t)seg * 2 * nv3;
        VH_HIP(hipMemcpyAsync(d.x, ck, nv3 * sizeof(double), hipMemcpyDeviceToDevice, s));
        VH_HIP(hipMemcpyAsync(d.v, ck + nv3, nv3 * sizeof(double), hipMemcpyDeviceToDevice, s));
        VH_HIP(vh::launch_refresh_u(d, s));
        // replay the segment, keeping x^(0) = y, x^(1), ..., x^(K) of every frame
        for (int32_t f = f0; f < f1; ++f) {
            double* itf = it + (size_t)(f - f0) * (K + 1) * nv3;
            VH_HIP(vh::launch_predictor(m->ls.predict, s));
            VH_HIP(hipMemcpyAsync(itf, d.x, nv3 * sizeof(double), hipMemcpyDeviceToDevice, s));
            for (int32_t k = 0; k < K; ++k) {
                VH_TRY(pd_iteration(nullptr, m->ls, s));
                VH_HIP(hipMemcpyAsync(itf + (size_t)(k + 1) * nv3, d.x, nv3 * sizeof(double),
                                      hipMemcpyDeviceToDevice, s));
            }
            VH_HIP(vh::launch_velocity(m->ls.velocity, s));
        }
        // reverse its frames
        for (int32_t f = f1 - 1; f >= f0; --f) {
            const double* itf = it + (size_t)(f - f0) * (K + 1) * nv3;
            VH_HIP(vh::launch_adj_frame(nf3, P.dt, true, xbar, vbar, xk, xn, ybar, s));
            for (int32_t k = K - 1; k >= 0; --k) {
                VH_HIP(hipMemcpyAsync(d.r, xk, (size_t)nf3 * sizeof(double), hipMemcpyDeviceToDevice, s));
                VH_TRY(solve(nullptr, m->ls, s, false, true));
                VH_HIP(hipMemcpyAsync(lam, d.delta, (size_t)nf3 * sizeof(double), hipMemcpyDeviceToDevice, s));
                VH_HIP(vh::launch_adj_local(G, d.nt, itf + (size_t)k * nv3, itf + (size_t)(k + 1) * nv3, lam, gbar,
                                            s));
                VH_HIP(vh::launch_adj_gather(G, d.n_free, lam, xk, ybar, s));
            }
            VH_HIP(vh::launch_adj_frame(nf3, P.dt, false, xbar, vbar, xk, xn, ybar, s));
        }
    }
    std::vector<double> g((size_t)d.nt);
    VH_HIP(hipMemcpyAsync(g.data(), gbar, g.size() * sizeof(double), hipMemcpyDeviceToHost, s));
    VH_HIP(hipStreamSynchronize(s));
    for (int32_t e = 0; e < d.nt; ++e) grad_gamma_s[P.elem_perm[e]] = g[e];
    uint32_t flags[4];
    VH_HIP(hipMemcpy(flags, d.flags, sizeof(flags), hipMemcpyDeviceToHost));
    if (flags[0]) return fail(VH_ENUMERIC, "non-finite value in the state");
    return VH_OK;
}

}  // extern "C"
