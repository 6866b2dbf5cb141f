// C ABI of libvhpd (declared in include/vhpd.h): handles, device buffers,
// the frame loop and the per-kernel test entry points.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "runtime.h"

namespace vhrt {

namespace {
thread_local std::string g_err;
}

int fail(int code, const std::string& msg) {
    g_err = msg;
    return code;
}

const char* last_error() { return g_err.c_str(); }

void charge(vh_ctx* ctx, size_t bytes) {
    ctx->in_use += bytes;
    ctx->peak = std::max(ctx->peak, ctx->in_use);
}

void uncharge(vh_ctx* ctx, size_t bytes) { ctx->in_use -= std::min(ctx->in_use, bytes); }

namespace {

void release_events(vh_mesh* m) {
    for (hipEvent_t e : m->ev_pool) (void)hipEventDestroy(e);
    m->ev_pool.clear();
    m->ev_used = 0;
    m->ev_pairs.clear();
}

// Records an event pair around a group of launches of one kernel class.
struct ProfScope {
    vh_mesh* m;
    hipStream_t s;
    int cls;
    size_t start = 0;
    bool on = false;
    hipError_t err = hipSuccess;
    hipEvent_t next() {
        if (m->ev_used == m->ev_pool.size()) {
            hipEvent_t e;
            err = hipEventCreate(&e);
            if (err != hipSuccess) return nullptr;
            m->ev_pool.push_back(e);
        }
        return m->ev_pool[m->ev_used++];
    }
    ProfScope(vh_mesh* m_, hipStream_t s_, int cls_) : m(m_), s(s_), cls(cls_) {
        on = m && ((m->prof_mask >> cls) & 1u);
        if (!on) return;
        start = m->ev_used;
        hipEvent_t e = next();
        if (e) err = hipEventRecord(e, s);
    }
    ~ProfScope() {
        if (!on || err != hipSuccess) return;
        hipEvent_t e = next();
        if (e && hipEventRecord(e, s) == hipSuccess) m->ev_pairs.push_back({start, cls});
    }
};

template <class T>
int dalloc(vh_mesh* m, T** p, size_t count) {
    size_t bytes = std::max<size_t>(count, 1) * sizeof(T);
    bytes = (bytes + 255) & ~(size_t)255;
    if (m->dry) {
        m->dry_bytes += bytes;
        *p = nullptr;
        return VH_OK;
    }
    if (m->ctx->budget && m->ctx->in_use + bytes > m->ctx->budget)
        return fail(VH_ENOMEM, "HBM budget exceeded");
    void* q = nullptr;
    hipError_t e = hipMalloc(&q, bytes);
    if (e != hipSuccess) return fail(VH_ENOMEM, std::string("hipMalloc: ") + hipGetErrorString(e));
    m->allocs.push_back(q);
    m->bytes += bytes;
    charge(m->ctx, bytes);
    *p = static_cast<T*>(q);
    return VH_OK;
}

template <class T>
int upload(vh_mesh* m, T** p, const std::vector<T>& v) {
    VH_TRY(dalloc(m, p, v.size()));
    if (!m->dry && !v.empty())
        VH_HIP(hipMemcpy(*p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice));
    return VH_OK;
}

// Allocates (or, in a dry run, counts) every device buffer of the plan and
// uploads the constant data; the state starts at rest.
int alloc_plan(vh_mesh* m) {
    const vh::Plan& P = m->plan;
    vh::DevMesh& d = m->dm;
    const size_t nv3 = (size_t)P.nv * 3;
    int r = VH_OK;
    auto chk = [&](int x) {
        if (r == VH_OK) r = x;
    };
    chk(upload(m, &d.X, P.X_int));
    chk(upload(m, &d.x, P.X_int));
    chk(dalloc(m, &d.v, nv3));
    chk(dalloc(m, &d.xprev, nv3));
    chk(dalloc(m, &d.y, nv3));
    chk(upload(m, &d.mass, P.mass_int));
    chk(upload(m, &d.perm, P.perm));
    chk(dalloc(m, &d.u, (size_t)P.nv));
    {
        std::vector<float4> tr;
        std::vector<uint2> lp;
        if (!m->dry) {
            tr.resize((size_t)P.nt * 4);
            std::memcpy(tr.data(), P.trec.data(), P.trec.size() * sizeof(float));
            lp.resize((size_t)P.nt);
            std::memcpy(lp.data(), P.lpos.data(), P.lpos.size() * sizeof(uint16_t));
            chk(upload(m, &d.trec, tr));
            chk(upload(m, &d.lpos, lp));
        } else {
            chk(dalloc(m, &d.trec, (size_t)P.nt * 4));
            chk(dalloc(m, &d.lpos, (size_t)P.nt));
        }
    }
    chk(upload(m, &d.blk_part, P.blk_part));
    chk(upload(m, &d.part_pack, P.part_pack));
    chk(dalloc(m, &d.part, (size_t)std::max<int32_t>(P.blk_part.back(), 1)));
    chk(upload(m, &d.vpart_ptr, P.vpart_ptr));
    chk(upload(m, &d.vpart, P.vpart));
    chk(dalloc(m, &d.r, (size_t)P.n_free * 3));
    chk(dalloc(m, &d.zf, (size_t)P.n_int * 3));
    chk(dalloc(m, &d.rg, (size_t)P.n_gamma * 3));
    chk(dalloc(m, &d.zg, (size_t)P.n_gamma * 3));
    chk(dalloc(m, &d.dg, (size_t)P.n_gamma * 3));
    chk(dalloc(m, &d.delta, (size_t)P.n_free * 3));
    chk(upload(m, &d.sub_off, P.sub_off));
    chk(upload(m, &d.chunks, P.chunks));
    chk(upload(m, &d.sub_fwd_ch, P.sub_fwd_ch));
    chk(upload(m, &d.sub_bwd_ch, P.sub_bwd_ch));
    chk(upload(m, &d.ivals, P.ivals));
    chk(upload(m, &d.bnd, P.bnd));
    chk(upload(m, &d.bnd_off, P.bnd_off));
    chk(upload(m, &d.dvals, P.dvals));
    chk(upload(m, &d.ctasks, P.ctasks));
    chk(upload(m, &d.cslots, P.cslots));
    chk(upload(m, &d.cgidx, P.cgidx));
    chk(dalloc(m, &d.cgf, (size_t)P.n_cgf * 3));
    chk(dalloc(m, &d.cgd, (size_t)P.n_cgd * 3));
    chk(upload(m, &d.K_ptr, P.K_ptr));
    chk(upload(m, &d.K_col, P.K_col));
    chk(upload(m, &d.K_val, P.K_val));
    chk(dalloc(m, &d.flags, 4));
    chk(dalloc(m, &d.regime, 8));
    const vh::CmsPlan& C = m->cms;
    if (C.modes > 0) {
        d.cms_modes = C.modes;
        d.cms_sweeps = C.sweeps;
        float *phi = nullptr, *psi = nullptr, *ilam = nullptr;
        int64_t *phi_off = nullptr, *psi_off = nullptr;
        double *invd = nullptr, *omega = nullptr;
        chk(upload(m, &phi, C.phi));
        chk(upload(m, &psi, C.psi));
        chk(upload(m, &ilam, C.ilam));
        chk(upload(m, &phi_off, C.phi_off));
        chk(upload(m, &psi_off, C.psi_off));
        chk(upload(m, &invd, C.inv_diag));
        if (C.sweeps > 0) chk(upload(m, &omega, C.omega));
        chk(dalloc(m, &d.cms_q, (size_t)P.D * C.modes * 3));
        chk(dalloc(m, &d.cms_b1, (size_t)P.n_free * 3));
        chk(dalloc(m, &d.cms_b2, (size_t)P.n_free * 3));
        d.cms_phi = phi;
        d.cms_psi = psi;
        d.cms_ilam = ilam;
        d.cms_phi_off = phi_off;
        d.cms_psi_off = psi_off;
        d.cms_invd = invd;
        d.cms_omega = omega;
    }
    return r;
}

// device bytes of the launch set of one garment alone: what build_launch_set
// allocates for it (one 16-byte table entry per block of each launch)
size_t launch_set_bytes(const vh::Plan& P) {
    size_t blocks = 2 * (size_t)vh::blocks_vertices(P.nv) + (size_t)vh::blocks_tets(P.nt) +
                    2 * (size_t)vh::blocks_vertices(P.n_free) + 2 * (size_t)P.D;
    for (const auto* ph : {&P.cfwd, &P.cbwd})
        for (const vh::CPhase& c : *ph) blocks += (size_t)vh::coarse_blocks(c.ntasks, c.group);
    return sizeof(vh::DevMesh) + sizeof(int32_t) * (4 * blocks + 1);
}

}  // namespace

int solve(vh_mesh* m, const LaunchSet& L, hipStream_t s, bool apply, bool keep_delta, const vh::DevMesh* G,
          bool resid) {
    {
        ProfScope ps(m, s, 3);
        VH_HIP(vh::launch_interior_fwd(with_record(L.ifwd, G), L.lds_fwd, s, resid));
    }
    {
        ProfScope ps(m, s, 4);
        for (const auto& c : L.cfwd) VH_HIP(vh::launch_coarse(with_record(c.ref, G), c.kind, c.group, s));
        for (const auto& c : L.cbwd) VH_HIP(vh::launch_coarse(with_record(c.ref, G), c.kind, c.group, s));
    }
    ProfScope ps(m, s, 5);
    if (L.cms_modes > 0) {
        // the inexact CMS solve: interiors from the modes, then the sweeps
        VH_HIP(vh::launch_cms_back(with_record(L.ibwd, G), L.lds_cms, L.cms_modes, s));
        VH_HIP(vh::launch_cms_iface(with_record(L.refine, G), s));
        for (int32_t k = 0; k < L.cms_sweeps; ++k) VH_HIP(vh::launch_cms_sweep(with_record(L.refine, G), k, s));
        VH_HIP(vh::launch_cms_apply(with_record(L.refine, G), L.cms_sweeps, apply, s));
        return VH_OK;
    }
    VH_HIP(vh::launch_interior_bwd(with_record(L.ibwd, G), L.lds_bwd, s, apply, keep_delta));
    return VH_OK;
}

int pd_iteration(vh_mesh* m, const LaunchSet& L, hipStream_t s, const vh::DevMesh* G) {
    {
        ProfScope ps(m, s, 1);
        VH_HIP(vh::launch_local(with_record(L.local, G), s, false));
    }
    // the residual r = b - L x is formed by the interior forward solve
    const bool refine = L.refine_steps > 0;
    VH_TRY(solve(m, L, s, true, refine, G, true));
    for (int32_t k = 0; k < L.refine_steps; ++k) {
        {
            ProfScope ps(m, s, 6);
            VH_HIP(vh::launch_refine_residual(with_record(L.refine, G), s));
        }
        VH_TRY(solve(m, L, s, true, k + 1 < L.refine_steps, G));
    }
    return VH_OK;
}

int check_ready(vh_mesh* m) {
    if (!m) return fail(VH_EINVAL, "null mesh");
    if (!m->factored) return fail(VH_ESTATE, "mesh is not prefactored");
    return VH_OK;
}

// check_ready plus: no server frames of this mesh pending
int check_quiet(vh_mesh* m) {
    VH_TRY(check_ready(m));
    return server_check_idle(m);
}

// check_ready plus: the mesh is not driven by the context's server (whose
// stream the caller's launches would not be ordered against)
int check_solo(vh_mesh* m) {
    VH_TRY(check_ready(m));
    if (m->srv_id >= 0 && m->ctx->srv)
        return fail(VH_ESTATE, "mesh is driven by the server; release it first");
    return VH_OK;
}

// user [nv][3] host -> internal device buffer (pinned rows: X or 0)
int put_user(vh_mesh* m, const double* host, double* dev_int, bool positions, hipStream_t s) {
    const vh::Plan& P = m->plan;
    std::vector<double>& st = m->stage;
    st.resize((size_t)P.nv * 3);
    for (int32_t i = 0; i < P.nv; ++i) {
        const int32_t u = P.perm[i];
        for (int c = 0; c < 3; ++c)
            st[3 * i + c] = (i < P.n_free) ? host[3 * u + c] : (positions ? P.X_int[3 * i + c] : 0.0);
    }
    VH_HIP(hipMemcpyAsync(dev_int, st.data(), st.size() * sizeof(double), hipMemcpyHostToDevice, s));
    VH_HIP(hipStreamSynchronize(s));
    return VH_OK;
}

namespace {

}  // namespace

int set_device(vh_mesh* m) {
    VH_HIP(hipSetDevice(m->ctx->device));
    return VH_OK;
}

void free_launch_set(vh_ctx* ctx, LaunchSet& L) {
    if (L.G) (void)hipFree(L.G);
    if (L.tables) (void)hipFree(L.tables);
    if (L.active) (void)hipFree(L.active);
    if (ctx) uncharge(ctx, L.bytes);
    L = LaunchSet();
}

void free_device(vh_mesh* m) {
    free_adjoint(m);
    free_embedding_device(m);
    if (m->gexec) {
        (void)hipGraphExecDestroy(m->gexec);
        m->gexec = nullptr;
    }
    free_launch_set(m->ctx, m->ls);
    for (void* p : m->allocs) (void)hipFree(p);
    m->allocs.clear();
    if (m->ctx) uncharge(m->ctx, m->bytes);
    m->bytes = 0;
    m->dm = vh::DevMesh();
    m->factored = false;
}

int build_launch_set(vh_ctx* ctx, const std::vector<vh_mesh*>& members, LaunchSet& L, bool check_budget) {
    free_launch_set(ctx, L);
    const int32_t ng = (int32_t)members.size();
    if (ng == 0) return fail(VH_EINVAL, "empty launch set");
    L.pd_iters = members[0]->plan.pd_iters;
    L.refine_steps = members[0]->refine;
    L.cms_modes = members[0]->cms.modes;
    L.cms_sweeps = members[0]->cms.sweeps;
    for (vh_mesh* m : members)
        if (m->cms.modes != L.cms_modes || m->cms.sweeps != L.cms_sweeps)
            return fail(VH_EINVAL, "garments in one batch need the same global solve (CMS modes and sweeps)");
    for (vh_mesh* m : members)
        if (m->plan.pd_iters != L.pd_iters || m->refine != L.refine_steps)
            return fail(VH_EINVAL, "garments in one batch need equal pd_iters and refine steps");
    std::vector<int32_t> tab;
    std::vector<std::pair<vh::LaunchRef*, size_t>> fix;   // ref -> table offset
    // per-garment blocks and parameters -> one table
    // one {garment, block within it, x0, x1} entry per block of the launch
    auto add = [&](vh::LaunchRef* ref, const std::vector<int32_t>& gids, const std::vector<int32_t>& nb,
                   const std::vector<int32_t>& x0, const std::vector<int32_t>& x1) {
        const size_t off = tab.size();   // a multiple of 4: entries stay 16-byte aligned
        int32_t acc = 0;
        for (size_t i = 0; i < gids.size(); ++i) {
            for (int32_t lb = 0; lb < nb[i]; ++lb) {
                const int32_t e[4] = {gids[i], lb, x0[i], x1[i]};
                tab.insert(tab.end(), e, e + 4);
            }
            acc += nb[i];
        }
        ref->nblocks = acc;
        fix.push_back({ref, off});
    };
    std::vector<int32_t> all(ng), zero(ng, 0), nb(ng);
    for (int32_t i = 0; i < ng; ++i) all[i] = i;
    auto per = [&](auto f) {
        for (int32_t i = 0; i < ng; ++i) nb[i] = f(members[i]->dm);
        return nb;
    };
    add(&L.predict, all, per([](const vh::DevMesh& d) { return vh::blocks_vertices(d.nv); }), zero, zero);
    add(&L.local, all, per([](const vh::DevMesh& d) { return vh::blocks_tets(d.nt); }), zero, zero);
    add(&L.residual, all, per([](const vh::DevMesh& d) { return vh::blocks_vertices(d.n_free); }), zero, zero);
    add(&L.refine, all, per([](const vh::DevMesh& d) { return vh::blocks_vertices(d.n_free); }), zero, zero);
    add(&L.velocity, all, per([](const vh::DevMesh& d) { return vh::blocks_vertices(d.nv); }), zero, zero);
    add(&L.ifwd, all, per([](const vh::DevMesh& d) { return d.D; }), zero, zero);
    add(&L.ibwd, all, per([](const vh::DevMesh& d) { return d.D; }), zero, zero);
    // interface phases: phase j of every garment whose phase j has the same
    // task kind and lane-group size goes into one launch; each garment's
    // phases stay in their order
    // (the launch list is complete before `add` keeps pointers into it)
    auto phases = [&](bool fwd, std::vector<CoarseLaunch>& out) {
        struct Pending {
            int32_t kind, grp;
            std::vector<int32_t> g, b, x0, x1;
        };
        std::vector<Pending> pend;
        size_t nj = 0;
        for (vh_mesh* m : members) nj = std::max(nj, (fwd ? m->plan.cfwd : m->plan.cbwd).size());
        for (size_t j = 0; j < nj; ++j)
            for (int32_t kind : {(int32_t)vh::PULLSUM, (int32_t)vh::GEMV, (int32_t)vh::BGEMV})
                for (int32_t grp : {16, 32, 64}) {
                    Pending p{kind, grp, {}, {}, {}, {}};
                    for (int32_t i = 0; i < ng; ++i) {
                        const auto& ph = fwd ? members[i]->plan.cfwd : members[i]->plan.cbwd;
                        if (j >= ph.size() || ph[j].group != grp || ph[j].kind != kind) continue;
                        p.g.push_back(i);
                        p.b.push_back(vh::coarse_blocks(ph[j].ntasks, grp));
                        p.x0.push_back(ph[j].task0);
                        p.x1.push_back(ph[j].ntasks);
                    }
                    if (!p.g.empty()) pend.push_back(std::move(p));
                }
        out.assign(pend.size(), CoarseLaunch{});
        for (size_t k = 0; k < pend.size(); ++k) {
            out[k].kind = pend[k].kind;
            out[k].group = pend[k].grp;
            add(&out[k].ref, pend[k].g, pend[k].b, pend[k].x0, pend[k].x1);
        }
    };
    phases(true, L.cfwd);
    phases(false, L.cbwd);
    // device copies
    std::vector<vh::DevMesh> G(ng);
    int32_t max_n = 1, max_nb = 0, max_cint = 0;
    for (int32_t i = 0; i < ng; ++i) {
        G[i] = members[i]->dm;
        max_n = std::max(max_n, G[i].max_sub_n);
        max_nb = std::max(max_nb, G[i].max_nb);
        max_cint = std::max(max_cint, G[i].max_cint);
    }
    // every garment of a launch carves LDS with its own sizes inside the batch maximum
    for (auto& d : G) {
        d.max_sub_n = max_n;
        d.max_nb = max_nb;
        d.max_cint = max_cint;
    }
    L.lds_fwd = vh::interior_fwd_lds(max_n, max_cint);
    L.lds_cms = vh::cms_back_lds(max_n, max_nb, L.cms_modes);
    L.lds_bwd = vh::interior_bwd_lds(max_n, max_nb);
    {
        int lds_limit = 0;
        VH_HIP(hipDeviceGetAttribute(&lds_limit, hipDeviceAttributeMaxSharedMemoryPerBlock, ctx->device));
        const size_t lds_need = std::max(L.lds_fwd, L.lds_bwd);
        if (lds_need > (size_t)lds_limit)
            return fail(VH_EINVAL, "a subdomain needs " + std::to_string(lds_need) + " bytes of LDS (limit " +
                                       std::to_string(lds_limit) + "); use more subdomains");
    }
    const size_t need = sizeof(vh::DevMesh) * ng + sizeof(int32_t) * (tab.size() + ng);
    if (check_budget && ctx->budget && ctx->in_use + need > ctx->budget)
        return fail(VH_ENOMEM, "HBM budget exceeded");
    L.ng = ng;
    VH_HIP(hipMalloc(&L.G, sizeof(vh::DevMesh) * ng));
    VH_HIP(hipMalloc(&L.tables, sizeof(int32_t) * tab.size()));
    VH_HIP(hipMalloc(&L.active, sizeof(int32_t) * ng));
    L.bytes = need;
    charge(ctx, need);
    VH_HIP(hipMemcpy(L.G, G.data(), sizeof(vh::DevMesh) * ng, hipMemcpyHostToDevice));
    VH_HIP(hipMemcpy(L.tables, tab.data(), sizeof(int32_t) * tab.size(), hipMemcpyHostToDevice));
    std::vector<int32_t> ones(ng, 1);
    VH_HIP(hipMemcpy(L.active, ones.data(), sizeof(int32_t) * ng, hipMemcpyHostToDevice));
    for (auto& f : fix) {
        f.first->G = L.G;
        f.first->L = L.tables + f.second;
        f.first->active = L.active;
    }
    return VH_OK;
}

int frame_direct(vh_mesh* m, const LaunchSet& L, hipStream_t s, const vh::DevMesh* G) {
    {
        ProfScope ps(m, s, 0);
        VH_HIP(vh::launch_predictor(with_record(L.predict, G), s));
    }
    for (int32_t k = 0; k < L.pd_iters; ++k) VH_TRY(pd_iteration(m, L, s, G));
    {
        ProfScope ps(m, s, 7);
        VH_HIP(vh::launch_velocity(with_record(L.velocity, G), s));
    }
    return VH_OK;
}

int capture_frame(const LaunchSet& L, hipStream_t* cap, hipGraphExec_t* out) {
    if (!*cap) VH_HIP(hipStreamCreateWithFlags(cap, hipStreamNonBlocking));
    VH_HIP(hipStreamBeginCapture(*cap, hipStreamCaptureModeThreadLocal));
    int rc = frame_direct(nullptr, L, *cap);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(*cap, &g);
    if (rc != VH_OK) {
        if (g) (void)hipGraphDestroy(g);
        return rc;
    }
    if (e != hipSuccess) return fail(VH_EDEVICE, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
    e = hipGraphInstantiate(out, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) {
        *out = nullptr;
        return fail(VH_EDEVICE, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
    }
    return VH_OK;
}

// Capture one frame (predictor, pd_iters x [local, residual, solve], velocity)
// into an executable graph on a private stream.
int ensure_graph(vh_mesh* m) {
    if (m->gexec) return VH_OK;
    return capture_frame(m->ls, &m->cap, &m->gexec);
}

int get_user(vh_mesh* m, const double* dev_int, double* host, int32_t rows, hipStream_t s) {
    const vh::Plan& P = m->plan;
    std::vector<double>& st = m->stage;
    st.resize((size_t)P.nv * 3);
    VH_HIP(hipMemcpyAsync(st.data(), dev_int, (size_t)rows * 3 * sizeof(double),
                          hipMemcpyDeviceToHost, s));
    VH_HIP(hipStreamSynchronize(s));
    std::fill(host, host + (size_t)P.nv * 3, 0.0);
    for (int32_t i = 0; i < rows; ++i) {
        const int32_t u = P.perm[i];
        for (int c = 0; c < 3; ++c) host[3 * u + c] = st[3 * i + c];
    }
    return VH_OK;
}

int host_factor(vh_mesh* m, int32_t n_subdomains, int32_t refine_steps) {
    if (!m->has_params) return fail(VH_ESTATE, "set_params must precede prefactor");
    if (refine_steps < 0) return fail(VH_EINVAL, "refine_steps must be >= 0");
    m->planned = false;
    std::string msg;
    vh::PlanOptions opt;
    opt.lanes32_min = m->ctx->cfg.iface_lanes32_min;
    opt.lanes64_min = m->ctx->cfg.iface_lanes64_min;
    opt.thin_separators = m->ctx->cfg.thin_separators != 0;
    opt.merge_max_cols = m->ctx->cfg.iface_merge_max_cols;
    opt.iface_on_device = true;
    int rc = vh::build_plan(m->X.data(), m->nv, m->tets.data(), m->nt, m->gs.data(), m->gv.data(),
                            m->mass.data(), m->pinned.data(), m->g, m->dt, m->iters, n_subdomains,
                            refine_steps, 32, vh::interior_chunk_words(), opt, m->plan, msg);
    if (rc != 0) return fail(rc, msg);
    // the interior kernels hold two LDS chunks (48 KB each) next to the
    // subdomain's vectors: gfx950 gives a workgroup up to 160 KB
    int lds_limit = 0;
    VH_HIP(hipDeviceGetAttribute(&lds_limit, hipDeviceAttributeMaxSharedMemoryPerBlock, m->ctx->device));
    const vh::Plan& P = m->plan;
    const size_t lds_need = std::max(vh::interior_fwd_lds(std::max(P.max_sub_n, 1), P.max_cint),
                                     vh::interior_bwd_lds(std::max(P.max_sub_n, 1), P.max_nb));
    if (lds_need > (size_t)lds_limit)
        return fail(VH_EINVAL, "a subdomain needs " + std::to_string(lds_need) + " bytes of LDS (limit " +
                                   std::to_string(lds_limit) + "); use more subdomains");
    m->cms = vh::CmsPlan();
    if (m->ctx->cfg.cms_modes > 0) {
        if (refine_steps > 0) return fail(VH_EINVAL, "the CMS solve is not combined with refinement steps");
        const size_t lc = vh::cms_back_lds(std::max(P.max_sub_n, 1), P.max_nb, m->ctx->cfg.cms_modes);
        if (lc > (size_t)lds_limit)
            return fail(VH_EINVAL, "a subdomain needs " + std::to_string(lc) + " bytes of LDS for the CMS solve");
        rc = vh::build_cms(P, m->ctx->cfg.cms_modes, m->ctx->cfg.cms_sweeps, m->cms, msg);
        if (rc != 0) return fail(rc, msg);
    }
    m->refine = refine_steps;
    m->planned = true;
    return VH_OK;
}

int device_need(vh_mesh* m, size_t* bytes) {
    if (!m->planned) return fail(VH_ESTATE, "mesh has no host factorization");
    m->dry = true;
    m->dry_bytes = 0;
    vh::DevMesh keep = m->dm;
    int rc = alloc_plan(m);
    m->dm = keep;
    m->dry = false;
    if (rc != VH_OK) return rc;
    *bytes = m->dry_bytes + launch_set_bytes(m->plan);
    return VH_OK;
}

int upload_device(vh_mesh* m) {
    if (!m->planned) return fail(VH_ESTATE, "mesh has no host factorization");
    VH_TRY(set_device(m));
    free_device(m);
    const vh::Plan& P = m->plan;
    vh::DevMesh& d = m->dm;
    d.nv = P.nv;
    d.nt = P.nt;
    d.n_free = P.n_free;
    d.n_int = P.n_int;
    d.n_gamma = P.n_gamma;
    d.D = P.D;
    d.max_sub_n = std::max(P.max_sub_n, 1);
    d.max_nb = P.max_nb;
    d.max_cint = P.max_cint;
    d.desc_table = m->ctx->cfg.interior_desc_table;
    d.dt = P.dt;
    for (int c = 0; c < 3; ++c) d.g[c] = P.gravity[c];
    int r = alloc_plan(m);
    if (r == VH_OK && !P.dvals_ready) r = device_interface_factor(m);
    if (r != VH_OK) {
        free_device(m);
        if (!m->plan.dvals_ready) m->planned = false;
        return r;
    }
    const size_t nv3 = (size_t)P.nv * 3;
    VH_HIP(hipMemset(d.v, 0, nv3 * sizeof(double)));
    VH_HIP(hipMemset(d.flags, 0, 4 * sizeof(uint32_t)));
    VH_HIP(hipMemset(d.regime, 0, 8 * sizeof(unsigned long long)));
    VH_HIP(hipMemset(d.delta, 0, (size_t)P.n_free * 3 * sizeof(double)));
    {
        std::vector<vh_mesh*> one{m};
        int lrc = build_launch_set(m->ctx, one, m->ls, true);
        if (lrc != VH_OK) {
            free_device(m);
            return lrc;
        }
    }
    VH_HIP(vh::launch_refresh_u(d, nullptr));
    VH_HIP(hipDeviceSynchronize());
    m->has_saved = false;
    m->factored = true;
    return VH_OK;
}

}  // namespace vhrt

using namespace vhrt;


extern "C" {

const char* vh_last_error(void) { return last_error(); }

int vh_ctx_create(vh_ctx** out, int device, size_t hbm_budget_bytes) {
    if (!out) return fail(VH_EINVAL, "null output handle");
    int n = 0;
    VH_HIP(hipGetDeviceCount(&n));
    if (device < 0 || device >= n) return fail(VH_EINVAL, "device id out of range");
    VH_HIP(hipSetDevice(device));
    // the interior solves may use up to the whole LDS of a workgroup: the
    // device limit is set once here (a kernel attribute of this device), so a
    // launch never depends on which meshes were prefactored before it
    int lds_limit = 0;
    VH_HIP(hipDeviceGetAttribute(&lds_limit, hipDeviceAttributeMaxSharedMemoryPerBlock, device));
    VH_HIP(vh::interior_set_lds_limit((size_t)lds_limit));
    vh_ctx* c = new vh_ctx();
    c->device = device;
    c->budget = hbm_budget_bytes;
    if (int rc = noalloc_init(c); rc != VH_OK) {
        delete c;
        return rc;
    }
    *out = c;
    return VH_OK;
}

int vh_ctx_get_config(const vh_ctx* ctx, vh_config* cfg) {
    if (!ctx || !cfg) return fail(VH_EINVAL, "null argument");
    *cfg = ctx->cfg;
    return VH_OK;
}

int vh_ctx_set_config(vh_ctx* ctx, const vh_config* cfg) {
    if (!ctx || !cfg) return fail(VH_EINVAL, "null argument");
    if (cfg->use_graphs != 0 && cfg->use_graphs != 1) return fail(VH_EINVAL, "use_graphs must be 0 or 1");
    if (cfg->iface_lanes32_min < 1 || cfg->iface_lanes64_min < 1)
        return fail(VH_EINVAL, "interface lane thresholds must be >= 1");
    if (cfg->thin_separators != 0 && cfg->thin_separators != 1)
        return fail(VH_EINVAL, "thin_separators must be 0 or 1");
    if (cfg->iface_merge_max_cols < 0) return fail(VH_EINVAL, "iface_merge_max_cols must be >= 0");
    if (cfg->cms_modes < 0 || cfg->cms_modes > 256 || cfg->cms_sweeps < 0 || cfg->cms_sweeps > 10000)
        return fail(VH_EINVAL, "cms_modes must be in 0..256 and cms_sweeps in 0..10000");
    if (cfg->interior_desc_table < 1 || cfg->interior_desc_table > 64)
        return fail(VH_EINVAL, "interior_desc_table must be in 1..64");
    ctx->cfg = *cfg;
    return VH_OK;
}

int vh_ctx_destroy(vh_ctx* ctx) {
    if (!ctx) return VH_OK;
    (void)hipSetDevice(ctx->device);
    server_destroy(ctx);
    std::vector<vh_mesh*> ms = ctx->meshes;
    for (vh_mesh* m : ms) vh_mesh_destroy(m);
    blas_destroy(ctx);
    delete ctx;
    return VH_OK;
}

int vh_ctx_set_hbm_budget(vh_ctx* ctx, size_t hbm_budget_bytes) {
    if (!ctx) return fail(VH_EINVAL, "null context");
    ctx->budget = hbm_budget_bytes;
    return VH_OK;
}

int vh_ctx_hbm_in_use(const vh_ctx* ctx, size_t* bytes) {
    if (!ctx || !bytes) return fail(VH_EINVAL, "null argument");
    *bytes = ctx->in_use;
    return VH_OK;
}

int vh_mesh_create(vh_ctx* ctx, vh_mesh** out, const double* rest_xyz, int32_t nv,
                   const int32_t* tets, int32_t nt) {
    if (!ctx || !out) return fail(VH_EINVAL, "null argument");
    std::string msg;
    if (vh::check_mesh(rest_xyz, nv, tets, nt, msg) != 0) return fail(VH_EINVAL, msg);
    vh_mesh* m = new vh_mesh();
    m->ctx = ctx;
    m->nv = nv;
    m->nt = nt;
    m->X.assign(rest_xyz, rest_xyz + (size_t)nv * 3);
    m->tets.assign(tets, tets + (size_t)nt * 4);
    ctx->meshes.push_back(m);
    *out = m;
    return VH_OK;
}

int vh_mesh_destroy(vh_mesh* m) {
    if (!m) return VH_OK;
    if (m->ctx && m->srv_id >= 0 && m->ctx->srv)
        return fail(VH_ESTATE, "mesh is still in the server; release it first");
    if (m->ctx) {
        (void)hipSetDevice(m->ctx->device);
        release_events(m);
        free_device(m);
        if (m->cap) (void)hipStreamDestroy(m->cap);
        auto& v = m->ctx->meshes;
        v.erase(std::remove(v.begin(), v.end(), m), v.end());
    }
    delete m;
    return VH_OK;
}

int vh_mesh_set_params(vh_mesh* m, const double* gamma_s, const double* gamma_v, const double* mass,
                       const uint8_t* pinned, const double* gravity, double dt, int32_t pd_iters) {
    if (!m || !gamma_s || !gamma_v || !mass || !pinned || !gravity)
        return fail(VH_EINVAL, "null argument");
    if (!(dt > 0.0) || !std::isfinite(dt)) return fail(VH_EINVAL, "dt must be positive");
    if (pd_iters < 1) return fail(VH_EINVAL, "pd_iters must be >= 1");
    for (int32_t e = 0; e < m->nt; ++e)
        if (!(gamma_s[e] >= 0.0) || !(gamma_v[e] >= 0.0) || !std::isfinite(gamma_s[e]) ||
            !std::isfinite(gamma_v[e]))
            return fail(VH_EINVAL, "gamma must be finite and >= 0 (element " + std::to_string(e) + ")");
    for (int32_t v = 0; v < m->nv; ++v)
        if (!pinned[v] && !(mass[v] > 0.0))
            return fail(VH_EINVAL, "mass must be > 0 on free vertex " + std::to_string(v));
    for (int c = 0; c < 3; ++c)
        if (!std::isfinite(gravity[c])) return fail(VH_EINVAL, "gravity must be finite");
    if (m->srv_id >= 0 && m->ctx->srv) return fail(VH_ESTATE, "mesh is in the server; release it first");
    if (m->factored) {
        (void)hipSetDevice(m->ctx->device);
        free_device(m);
    }
    m->planned = false;
    m->has_saved = false;
    m->gs.assign(gamma_s, gamma_s + m->nt);
    m->gv.assign(gamma_v, gamma_v + m->nt);
    m->mass.assign(mass, mass + m->nv);
    m->pinned.assign(pinned, pinned + m->nv);
    for (int c = 0; c < 3; ++c) m->g[c] = gravity[c];
    m->dt = dt;
    m->iters = pd_iters;
    m->has_params = true;
    return VH_OK;
}

int vh_mesh_prefactor(vh_mesh* m, int32_t n_subdomains, int32_t refine_steps, int32_t precision_mode) {
    if (!m) return fail(VH_EINVAL, "null mesh");
    if (precision_mode != VH_PRECISION_MIXED) return fail(VH_EINVAL, "unknown precision_mode");
    if (m->srv_id >= 0 && m->ctx->srv) return fail(VH_ESTATE, "mesh is in the server; release it first");
    VH_TRY(set_device(m));
    free_device(m);
    VH_TRY(host_factor(m, n_subdomains, refine_steps));
    return upload_device(m);
}

int vh_mesh_refactor(vh_mesh* m, const double* gamma_s, const double* gamma_v) {
    VH_TRY(check_solo(m));
    if (!gamma_s || !gamma_v) return fail(VH_EINVAL, "null argument");
    for (int32_t e = 0; e < m->nt; ++e)
        if (!(gamma_s[e] >= 0.0) || !(gamma_v[e] >= 0.0) || !std::isfinite(gamma_s[e]) ||
            !std::isfinite(gamma_v[e]))
            return fail(VH_EINVAL, "gamma must be finite and >= 0 (element " + std::to_string(e) + ")");
    if (m->cms.modes > 0) return fail(VH_EINVAL, "a mesh with the CMS solve is refactored by vh_mesh_prefactor");
    VH_TRY(set_device(m));
    std::string msg;
    const int rc = vh::refactor_plan(m->plan, m->X.data(), m->tets.data(), gamma_s, gamma_v, msg);
    if (rc != 0) {
        // the host plan holds a partial factorization
        free_device(m);
        m->planned = false;
        return fail(rc, msg);
    }
    m->gs.assign(gamma_s, gamma_s + m->nt);
    m->gv.assign(gamma_v, gamma_v + m->nt);
    // the values in place: same sizes and addresses (work in flight finishes first)
    const vh::Plan& P = m->plan;
    const vh::DevMesh& d = m->dm;
    VH_HIP(hipDeviceSynchronize());
    VH_HIP(hipMemcpy(d.trec, P.trec.data(), P.trec.size() * sizeof(float), hipMemcpyHostToDevice));
    VH_HIP(hipMemcpy(d.ivals, P.ivals.data(), P.ivals.size() * sizeof(float), hipMemcpyHostToDevice));
    VH_HIP(hipMemcpy(d.K_val, P.K_val.data(), P.K_val.size() * sizeof(double), hipMemcpyHostToDevice));
    free_adjoint(m);
    if (P.dvals_ready) {
        VH_HIP(hipMemcpy(d.dvals, P.dvals.data(), P.dvals.size() * sizeof(double), hipMemcpyHostToDevice));
    } else {
        const int frc = device_interface_factor(m);   // the interface factor on the device, in place
        if (frc != VH_OK) {
            free_device(m);
            m->planned = false;
            return frc;
        }
    }
    return VH_OK;
}

int vh_mesh_step(vh_mesh* m, int32_t n_frames, void* stream) {
    VH_TRY(check_solo(m));
    if (n_frames < 0) return fail(VH_EINVAL, "n_frames must be >= 0");
    VH_TRY(set_device(m));
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (m->prof_mask || !m->ctx->cfg.use_graphs) {
        for (int32_t f = 0; f < n_frames; ++f) VH_TRY(frame_direct(m, m->ls, s));
        return VH_OK;
    }
    if (n_frames > 0) VH_TRY(ensure_graph(m));
    for (int32_t f = 0; f < n_frames; ++f) VH_HIP(hipGraphLaunch(m->gexec, s));
    return VH_OK;
}

int vh_mesh_read_state(vh_mesh* m, double* x, double* v, void* stream) {
    if (!m) return fail(VH_EINVAL, "null mesh");
    if (!x && !v) return fail(VH_EINVAL, "null output arrays");
    if (!m->factored && m->has_saved) {
        if (x) std::copy(m->saved_x.begin(), m->saved_x.end(), x);
        if (v) std::copy(m->saved_v.begin(), m->saved_v.end(), v);
        return VH_OK;
    }
    VH_TRY(check_quiet(m));
    VH_TRY(set_device(m));
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (x) VH_TRY(get_user(m, m->dm.x, x, m->plan.nv, s));
    if (v) VH_TRY(get_user(m, m->dm.v, v, m->plan.nv, s));
    uint32_t flags[4];
    VH_HIP(hipMemcpy(flags, m->dm.flags, sizeof(flags), hipMemcpyDeviceToHost));
    if (flags[0]) return fail(VH_ENUMERIC, "non-finite value in the state");
    return VH_OK;
}

int vh_mesh_write_state(vh_mesh* m, const double* x, const double* v, void* stream) {
    VH_TRY(check_quiet(m));
    if (!x || !v) return fail(VH_EINVAL, "null input arrays");
    VH_TRY(set_device(m));
    hipStream_t s = static_cast<hipStream_t>(stream);
    VH_TRY(put_user(m, x, m->dm.x, true, s));
    VH_TRY(put_user(m, v, m->dm.v, false, s));
    VH_HIP(vh::launch_refresh_u(m->dm, s));
    VH_HIP(hipMemsetAsync(m->dm.flags, 0, sizeof(uint32_t), s));
    VH_HIP(hipStreamSynchronize(s));
    return VH_OK;
}

int vh_mesh_read_state_device(vh_mesh* m, double* x_dev, double* v_dev, void* stream) {
    VH_TRY(check_quiet(m));
    VH_TRY(set_device(m));
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (x_dev) VH_HIP(vh::launch_to_user(m->dm.nv, m->dm.perm, m->dm.x, x_dev, s));
    if (v_dev) VH_HIP(vh::launch_to_user(m->dm.nv, m->dm.perm, m->dm.v, v_dev, s));
    if (m->srv_id >= 0) VH_HIP(hipStreamSynchronize(s));   // ordered before the server's next frame
    return VH_OK;
}

int vh_mesh_write_state_device(vh_mesh* m, const double* x_dev, const double* v_dev, void* stream) {
    VH_TRY(check_quiet(m));
    if (!x_dev || !v_dev) return fail(VH_EINVAL, "null input arrays");
    VH_TRY(set_device(m));
    hipStream_t s = static_cast<hipStream_t>(stream);
    VH_HIP(vh::launch_from_user(m->dm.nv, m->dm.n_free, m->dm.perm, x_dev, m->dm.X, m->dm.x, s));
    VH_HIP(vh::launch_from_user(m->dm.nv, m->dm.n_free, m->dm.perm, v_dev, nullptr, m->dm.v, s));
    VH_HIP(vh::launch_refresh_u(m->dm, s));
    if (m->srv_id >= 0) VH_HIP(hipStreamSynchronize(s));   // ordered before the server's next frame
    return VH_OK;
}

int vh_mesh_regime_counts(vh_mesh* m, vh_regime_counts* out, int32_t reset, void* stream) {
    if (!m || !out) return fail(VH_EINVAL, "null argument");
    VH_TRY(check_quiet(m));
    VH_TRY(set_device(m));
    hipStream_t s = static_cast<hipStream_t>(stream);
    unsigned long long c[8];
    VH_HIP(hipMemcpyAsync(c, m->dm.regime, sizeof(c), hipMemcpyDeviceToHost, s));
    VH_HIP(hipStreamSynchronize(s));
    out->clamped = c[0];
    out->inverted = c[1];
    out->det_ge2 = c[2];
    out->squash = c[3];
    out->no_plus_root = c[4];
    if (reset) {
        VH_HIP(hipMemsetAsync(m->dm.regime, 0, sizeof(c), s));
        VH_HIP(hipStreamSynchronize(s));
    }
    return VH_OK;
}

int vh_mesh_get_info(const vh_mesh* m, vh_mesh_info* info) {
    if (!m || !info) return fail(VH_EINVAL, "null argument");
    if (!m->factored) return fail(VH_ESTATE, "mesh is not prefactored");
    const vh::Plan& P = m->plan;
    info->nv = P.nv;
    info->nt = P.nt;
    info->n_free = P.n_free;
    info->n_interior = P.n_int;
    info->n_interface = P.n_gamma;
    info->n_subdomains = P.D;
    info->n_supernodes = (int32_t)P.sn.size();
    info->n_coarse_levels = P.n_clevels;
    info->max_interior_phases = P.max_sub_phases;
    info->nnz_interior = P.nnz_int;
    info->nnz_coarse = P.nnz_coarse;
    info->device_bytes = m->bytes;
    info->prefactor_seconds = P.seconds;
    info->n_partials = P.blk_part.empty() ? 0 : P.blk_part.back();
    const int64_t npart = info->n_partials, nblk = (int64_t)P.blk_part.size();
    info->bytes_local = (int64_t)P.nt * (64 + 8) + (int64_t)P.nv * 16 + npart * (4 + 16) + nblk * 4;
    info->bytes_residual = (int64_t)P.n_free * (4 + 8 + 24 + 24 + 24) + 4 + npart * (4 + 16);
    int64_t fw = 0, bw = 0;
    for (int32_t c = P.sub_fwd_ch[0]; c < P.sub_fwd_ch[P.D]; ++c) fw += 4 * (int64_t)P.chunks[c].nv + 32;
    for (int32_t c = P.sub_bwd_ch[0]; c < P.sub_bwd_ch[P.D]; ++c) bw += 4 * (int64_t)P.chunks[c].nv + 32;
    // forward: chunks, r in, z out, interface contributions out
    info->bytes_interior_fwd = fw + (int64_t)P.n_int * (24 + 12) + (int64_t)P.n_cgf * 12;
    // backward: chunks, z in, boundary values in, x/X in, x/u out (interior and interface rows)
    info->bytes_interior_bwd = bw + (int64_t)P.n_int * 12 + (int64_t)P.bnd.size() * 24 +
                               (int64_t)P.n_free * (24 + 24 + 24 + 16) + (int64_t)P.n_gamma * 24;
    // interface: every FP64 value once (forward rows, backward columns), task
    // descriptors, slot and gather lists, contributions in/out, r/z/d vectors
    info->bytes_interface = 8 * (int64_t)P.dvals.size() + 32 * (int64_t)P.ctasks.size() +
                            4 * (int64_t)(P.cslots.size() + P.cgidx.size()) + (int64_t)P.n_cgf * 12 +
                            (int64_t)P.n_cgd * 24 * 2 + (int64_t)P.n_gamma * 24 * 5;
    info->interface_launches = (int32_t)(P.cfwd.size() + P.cbwd.size());
    return VH_OK;
}

int vh_debug_local_step(vh_mesh* m, const double* x, double* T, double* sigma, double* s_out) {
    VH_TRY(check_solo(m));
    if (!x || !T) return fail(VH_EINVAL, "null argument");
    VH_TRY(set_device(m));
    vh::DevMesh& d = m->dm;
    const int32_t nt = d.nt;
    if (!d.dbg_T) {
        VH_TRY(dalloc(m, &d.dbg_T, (size_t)nt * 9));
        VH_TRY(dalloc(m, &d.dbg_sig, (size_t)nt * 3));
        VH_TRY(dalloc(m, &d.dbg_s, (size_t)nt * 3));
    }
    VH_TRY(put_user(m, x, d.x, true, nullptr));
    VH_HIP(hipMemcpy(&m->ls.G[0].dbg_T, &d.dbg_T, 3 * sizeof(float*), hipMemcpyHostToDevice));
    VH_HIP(vh::launch_refresh_u(d, nullptr));
    VH_HIP(vh::launch_local(m->ls.local, nullptr, true));
    VH_HIP(hipDeviceSynchronize());
    std::vector<float> hT((size_t)nt * 9), hs((size_t)nt * 3), hss((size_t)nt * 3);
    VH_HIP(hipMemcpy(hT.data(), d.dbg_T, hT.size() * 4, hipMemcpyDeviceToHost));
    VH_HIP(hipMemcpy(hs.data(), d.dbg_sig, hs.size() * 4, hipMemcpyDeviceToHost));
    VH_HIP(hipMemcpy(hss.data(), d.dbg_s, hss.size() * 4, hipMemcpyDeviceToHost));
    const auto& ep = m->plan.elem_perm;
    for (int32_t e = 0; e < nt; ++e) {
        const int32_t u = ep[e];
        for (int k = 0; k < 9; ++k) T[(size_t)u * 9 + k] = hT[(size_t)e * 9 + k];
        for (int k = 0; k < 3; ++k) {
            if (sigma) sigma[(size_t)u * 3 + k] = hs[(size_t)e * 3 + k];
            if (s_out) s_out[(size_t)u * 3 + k] = hss[(size_t)e * 3 + k];
        }
    }
    return VH_OK;
}

int vh_debug_scatter_colored(vh_mesh* m, const double* x, double* f, int32_t* n_colors) {
    VH_TRY(check_solo(m));
    if (!x || !f) return fail(VH_EINVAL, "null argument");
    VH_TRY(set_device(m));
    vh::DevMesh& d = m->dm;
    const vh::Plan& P = m->plan;
    const int32_t nt = d.nt, nf = d.n_free;
    // greedy colouring in element order: the smallest colour no tet sharing a
    // free vertex has taken yet (one bit per colour and vertex)
    std::vector<uint64_t> used((size_t)P.nv, 0);
    std::vector<int32_t> colour((size_t)nt);
    int32_t ncol = 0;
    for (int32_t e = 0; e < nt; ++e) {
        uint64_t forbidden = 0;
        for (int a = 0; a < 4; ++a) {
            const int32_t v = P.tet_soa[(size_t)a * nt + e];
            if (v < nf) forbidden |= used[v];
        }
        if (~forbidden == 0) return fail(VH_EINVAL, "the element colouring needs more than 64 colours");
        const int32_t c = __builtin_ctzll(~forbidden);
        colour[e] = c;
        ncol = std::max(ncol, c + 1);
        for (int a = 0; a < 4; ++a) {
            const int32_t v = P.tet_soa[(size_t)a * nt + e];
            if (v < nf) used[v] |= (uint64_t)1 << c;
        }
    }
    std::vector<int32_t> ptr(ncol + 1, 0), list((size_t)nt);
    for (int32_t e = 0; e < nt; ++e) ++ptr[colour[e] + 1];
    for (int32_t c = 0; c < ncol; ++c) ptr[c + 1] += ptr[c];
    {
        std::vector<int32_t> fill(ptr.begin(), ptr.end() - 1);
        for (int32_t e = 0; e < nt; ++e) list[fill[colour[e]]++] = e;
    }
    if (!d.dbg_T) {
        VH_TRY(dalloc(m, &d.dbg_T, (size_t)nt * 9));
        VH_TRY(dalloc(m, &d.dbg_sig, (size_t)nt * 3));
        VH_TRY(dalloc(m, &d.dbg_s, (size_t)nt * 3));
    }
    if (!d.dbg_col) {
        VH_TRY(dalloc(m, &d.dbg_col, (size_t)nt));
        VH_TRY(dalloc(m, &d.dbg_b, (size_t)nf * 3));
    }
    VH_TRY(put_user(m, x, d.x, true, nullptr));
    VH_HIP(hipMemcpy(&m->ls.G[0].dbg_T, &d.dbg_T, 3 * sizeof(float*), hipMemcpyHostToDevice));
    VH_HIP(vh::launch_refresh_u(d, nullptr));
    VH_HIP(vh::launch_local(m->ls.local, nullptr, true));
    VH_HIP(hipMemcpy(d.dbg_col, list.data(), list.size() * sizeof(int32_t), hipMemcpyHostToDevice));
    VH_HIP(hipMemset(d.dbg_b, 0, (size_t)nf * 3 * sizeof(float)));
    for (int32_t c = 0; c < ncol; ++c)
        VH_HIP(vh::launch_scatter_colour(d, d.dbg_col + ptr[c], ptr[c + 1] - ptr[c], nullptr));
    VH_HIP(hipDeviceSynchronize());
    std::vector<float> hb((size_t)nf * 3);
    VH_HIP(hipMemcpy(hb.data(), d.dbg_b, hb.size() * sizeof(float), hipMemcpyDeviceToHost));
    std::fill(f, f + (size_t)P.nv * 3, 0.0);
    for (int32_t i = 0; i < nf; ++i)
        for (int c = 0; c < 3; ++c) f[3 * (size_t)P.perm[i] + c] = hb[3 * (size_t)i + c];
    if (n_colors) *n_colors = ncol;
    return VH_OK;
}

namespace {
int debug_residual(vh_mesh* m, const double* x, const double* y, double* r, bool in_solve) {
    VH_TRY(check_solo(m));
    if (!x || !y || !r) return fail(VH_EINVAL, "null argument");
    VH_TRY(set_device(m));
    vh::DevMesh& d = m->dm;
    VH_TRY(put_user(m, x, d.x, true, nullptr));
    VH_TRY(put_user(m, y, d.y, true, nullptr));
    VH_HIP(vh::launch_refresh_u(d, nullptr));
    VH_HIP(vh::launch_local(m->ls.local, nullptr, false));
    if (in_solve) VH_HIP(vh::launch_interior_fwd(m->ls.ifwd, m->ls.lds_fwd, nullptr, true));
    else VH_HIP(vh::launch_residual(m->ls.residual, nullptr));
    VH_HIP(hipDeviceSynchronize());
    return get_user(m, d.r, r, d.n_free, nullptr);
}
}  // namespace

int vh_debug_residual(vh_mesh* m, const double* x, const double* y, double* r) {
    return debug_residual(m, x, y, r, false);
}

int vh_debug_residual_in_solve(vh_mesh* m, const double* x, const double* y, double* r) {
    return debug_residual(m, x, y, r, true);
}

int vh_debug_interface_factor(vh_mesh* m, double* out, int64_t* count) {
    VH_TRY(check_solo(m));
    if (!count) return fail(VH_EINVAL, "null argument");
    const int64_t n = (int64_t)m->plan.dvals.size();
    if (!out) {
        *count = n;
        return VH_OK;
    }
    if (*count != n) return fail(VH_EINVAL, "count must equal the number of interface factor values");
    VH_TRY(set_device(m));
    VH_HIP(hipDeviceSynchronize());
    if (n > 0) VH_HIP(hipMemcpy(out, m->dm.dvals, (size_t)n * sizeof(double), hipMemcpyDeviceToHost));
    return VH_OK;
}

int vh_debug_solve(vh_mesh* m, const double* rhs, double* out) {
    VH_TRY(check_solo(m));
    if (!rhs || !out) return fail(VH_EINVAL, "null argument");
    VH_TRY(set_device(m));
    vh::DevMesh& d = m->dm;
    const vh::Plan& P = m->plan;
    std::vector<double> st((size_t)P.n_free * 3);
    for (int32_t i = 0; i < P.n_free; ++i)
        for (int c = 0; c < 3; ++c) st[3 * i + c] = rhs[3 * P.perm[i] + c];
    VH_HIP(hipMemcpy(d.r, st.data(), st.size() * sizeof(double), hipMemcpyHostToDevice));
    VH_TRY(solve(m, m->ls, nullptr, false, true));
    VH_HIP(hipDeviceSynchronize());
    return get_user(m, d.delta, out, d.n_free, nullptr);
}

int vh_mesh_time_kernel(vh_mesh* m, int32_t kernel_class, int32_t reps, void* stream) {
    VH_TRY(check_solo(m));
    if (reps < 1) return fail(VH_EINVAL, "reps must be >= 1");
    VH_TRY(set_device(m));
    hipStream_t s = static_cast<hipStream_t>(stream);
    for (int32_t r = 0; r < reps; ++r) {
        switch (kernel_class) {
            case 1: VH_HIP(vh::launch_local(m->ls.local, s, false)); break;
            case 2: VH_HIP(vh::launch_residual(m->ls.residual, s)); break;
            case 3: VH_HIP(vh::launch_interior_fwd(m->ls.ifwd, m->ls.lds_fwd, s, true)); break;
            case 4:
                for (const auto& c : m->ls.cfwd) VH_HIP(vh::launch_coarse(c.ref, c.kind, c.group, s));
                for (const auto& c : m->ls.cbwd) VH_HIP(vh::launch_coarse(c.ref, c.kind, c.group, s));
                break;
            case 5: VH_HIP(vh::launch_interior_bwd(m->ls.ibwd, m->ls.lds_bwd, s, false, false)); break;
            case 6: VH_HIP(vh::launch_interior_fwd(m->ls.ifwd, m->ls.lds_fwd, s, false)); break;
            default: return fail(VH_EINVAL, "kernel_class must be 1..6");
        }
    }
    return VH_OK;
}

int vh_mesh_profile(vh_mesh* m, uint32_t class_mask) {
    VH_TRY(check_solo(m));
    VH_TRY(set_device(m));
    m->prof_mask = class_mask & 0xFFu;
    m->ev_used = 0;
    m->ev_pairs.clear();
    return VH_OK;
}

int vh_mesh_profile_read(vh_mesh* m, double* ms, int64_t* launches) {
    VH_TRY(check_ready(m));
    if (!ms || !launches) return fail(VH_EINVAL, "null argument");
    VH_TRY(set_device(m));
    for (int c = 0; c < VH_PROFILE_CLASSES; ++c) {
        ms[c] = 0.0;
        launches[c] = 0;
    }
    for (const auto& pr : m->ev_pairs) {
        VH_HIP(hipEventSynchronize(m->ev_pool[pr.first + 1]));
        float t = 0.0f;
        VH_HIP(hipEventElapsedTime(&t, m->ev_pool[pr.first], m->ev_pool[pr.first + 1]));
        ms[pr.second] += t;
        launches[pr.second] += 1;
    }
    m->ev_used = 0;
    m->ev_pairs.clear();
    return VH_OK;
}

}  // extern "C"
