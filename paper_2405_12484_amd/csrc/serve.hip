// Step server of a context: garments wait for device memory in FIFO order,
// step requests are queued per garment, and each launch runs one frame of
// every resident garment that has a request waiting (continuous batching).
//
// A batched launch replays one captured frame graph over all resident
// garments; a per-garment flag array, copied in before the replay, masks off
// the garments without a request, so the graph stays valid until the set of
// resident garments changes.  Every garment is computed by the same blocks,
// in the same order, alone or in any mix (a block reads its own garment's
// descriptor only), so its trajectory does not depend on the mix.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <deque>
#include <string>
#include <vector>

#include "runtime.h"
#include "serve_policy.h"

namespace vhrt {

struct Batch {
    std::vector<int32_t> ids;   // garments stepped by this launch
    hipEvent_t done = nullptr;
};

struct Server {
    int32_t mode = VH_SERVE_BATCHED;
    int32_t depth = 2;              // launches enqueued ahead of the GPU
    int32_t max_batch = 0;          // garments per launch, 0 = no limit
    int32_t pd_iters = -1, refine = -1;
    int32_t max_n = 1, max_nb = 0, max_cint = 0;   // LDS sizes over every garment added
    vh::ServePolicy pol;
    std::vector<vh_mesh*> mesh;     // garment id -> mesh (null once released)
    std::vector<uint8_t> release_req;
    hipStream_t s = nullptr;
    // the batched frame over the resident garments
    LaunchSet ls;
    std::vector<int32_t> pos;       // garment id -> position in ls (-1: not in it)
    hipStream_t cap = nullptr;
    hipGraphExec_t gexec = nullptr;
    bool dirty = true;              // resident set changed since ls was built
    bool use_graph = true;
    int32_t* h_active = nullptr;    // pinned [depth][ls.ng] flag slots
    int32_t next_slot = 0;
    std::deque<Batch> inflight;
    std::vector<hipEvent_t> ev_free;
    hipEvent_t ev0 = nullptr;       // clock origin on the GPU
    std::chrono::steady_clock::time_point t0;
    int64_t launches = 0, garment_frames = 0;
};

namespace {

double host_now(const Server& S) {
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - S.t0).count();
}

int free_batched(vh_ctx* ctx, Server& S) {
    if (S.gexec) {
        (void)hipGraphExecDestroy(S.gexec);
        S.gexec = nullptr;
    }
    free_launch_set(ctx, S.ls);
    if (S.h_active) {
        (void)hipHostFree(S.h_active);
        S.h_active = nullptr;
    }
    std::fill(S.pos.begin(), S.pos.end(), -1);
    return VH_OK;
}

// Retire completed launches, oldest first; with block, wait for the oldest.
int retire(Server& S, bool block) {
    while (!S.inflight.empty()) {
        Batch& B = S.inflight.front();
        hipError_t e = block ? hipEventSynchronize(B.done) : hipEventQuery(B.done);
        if (e == hipErrorNotReady) break;
        if (e != hipSuccess) return fail(VH_EDEVICE, std::string("server launch: ") + hipGetErrorString(e));
        float ms = 0.0f;
        VH_HIP(hipEventElapsedTime(&ms, S.ev0, B.done));
        S.pol.complete(B.ids, 1e-3 * (double)ms);
        S.ev_free.push_back(B.done);
        S.inflight.pop_front();
        block = false;
    }
    return VH_OK;
}

int drain(Server& S) {
    while (!S.inflight.empty()) VH_TRY(retire(S, true));
    return VH_OK;
}

// Frees a released garment's device memory once it has nothing outstanding,
// keeping its last state on the host.
int apply_releases(vh_ctx* ctx, Server& S) {
    for (int32_t g = 0; g < (int32_t)S.mesh.size(); ++g) {
        if (!S.release_req[g] || !S.pol.idle(g)) continue;
        vh_mesh* m = S.mesh[g];
        S.release_req[g] = 0;
        S.pol.release(g);
        S.mesh[g] = nullptr;
        m->srv_id = -1;
        if (m->factored) {
            VH_TRY(set_device(m));
            m->saved_x.assign((size_t)m->nv * 3, 0.0);
            m->saved_v.assign((size_t)m->nv * 3, 0.0);
            VH_TRY(get_user(m, m->dm.x, m->saved_x.data(), m->plan.nv, S.s));
            VH_TRY(get_user(m, m->dm.v, m->saved_v.data(), m->plan.nv, S.s));
            // launches still queued never touch it: its flag stays 0 in every slot
            free_device(m);
            m->has_saved = true;
        }
        if (S.pos[g] >= 0) S.pos[g] = -1;
        (void)ctx;
    }
    return VH_OK;
}

// Admits queued garments in FIFO order while they fit the budget; each one's
// own frame graph (used when it runs alone) is captured now.
int admit(vh_ctx* ctx, Server& S) {
    for (int32_t g : S.pol.to_admit(ctx->in_use, ctx->budget)) {
        vh_mesh* m = S.mesh[g];
        VH_TRY(upload_device(m));
        if (m->ctx->cfg.use_graphs) VH_TRY(ensure_graph(m));
        S.pol.admit(g);
        S.dirty = true;
    }
    return VH_OK;
}

// Rebuild the batched launch set and its graph over the resident garments.
int rebuild(vh_ctx* ctx, Server& S) {
    VH_TRY(drain(S));
    VH_TRY(free_batched(ctx, S));
    std::vector<vh_mesh*> members;
    for (int32_t g = 0; g < (int32_t)S.mesh.size(); ++g)
        if (S.mesh[g] && S.pol.state(g) == vh::ServePolicy::RESIDENT) {
            S.pos[g] = (int32_t)members.size();
            members.push_back(S.mesh[g]);
        }
    S.dirty = false;
    if (members.empty()) return VH_OK;
    VH_TRY(build_launch_set(ctx, members, S.ls, false));
    VH_HIP(hipHostMalloc(reinterpret_cast<void**>(&S.h_active), sizeof(int32_t) * S.ls.ng * S.depth,
                         hipHostMallocDefault));
    std::fill(S.h_active, S.h_active + (size_t)S.ls.ng * S.depth, 0);
    S.next_slot = 0;
    if (S.use_graph) VH_TRY(capture_frame(S.ls, &S.cap, &S.gexec));
    return VH_OK;
}

int take_event(Server& S, hipEvent_t* e) {
    if (!S.ev_free.empty()) {
        *e = S.ev_free.back();
        S.ev_free.pop_back();
        return VH_OK;
    }
    VH_HIP(hipEventCreate(e));
    return VH_OK;
}

// One frame of garments `ids`.  A single garment runs its own frame graph
// (its launches cover only its blocks); several run the batched graph with
// the others masked off.  Both compute every garment identically.
int launch(Server& S, const std::vector<int32_t>& ids) {
    if (S.mode == VH_SERVE_SEQUENTIAL || ids.size() == 1) {
        vh_mesh* m = S.mesh[ids[0]];
        if (m->ctx->cfg.use_graphs) {
            VH_TRY(ensure_graph(m));
            VH_HIP(hipGraphLaunch(m->gexec, S.s));
        } else {
            VH_TRY(frame_direct(nullptr, m->ls, S.s));
        }
    } else {
        // this slot's previous copy is complete: its launch was retired before
        // fewer than `depth` launches were in flight
        int32_t* h = S.h_active + (size_t)S.next_slot * S.ls.ng;
        S.next_slot = (S.next_slot + 1) % S.depth;
        std::fill(h, h + S.ls.ng, 0);
        for (int32_t g : ids) h[S.pos[g]] = 1;
        VH_HIP(hipMemcpyAsync(S.ls.active, h, sizeof(int32_t) * S.ls.ng, hipMemcpyHostToDevice, S.s));
        if (S.gexec)
            VH_HIP(hipGraphLaunch(S.gexec, S.s));
        else
            VH_TRY(frame_direct(nullptr, S.ls, S.s));
    }
    Batch B;
    B.ids = ids;
    VH_TRY(take_event(S, &B.done));
    VH_HIP(hipEventRecord(B.done, S.s));
    S.pol.launch(ids);
    S.inflight.push_back(std::move(B));
    S.launches += 1;
    S.garment_frames += (int64_t)ids.size();
    return VH_OK;
}

int tick(vh_ctx* ctx, Server& S, bool wait, int32_t* n_launched) {
    int32_t n = 0;
    VH_TRY(retire(S, false));
    VH_TRY(apply_releases(ctx, S));
    VH_TRY(admit(ctx, S));
    if (S.mode == VH_SERVE_BATCHED && S.dirty) VH_TRY(rebuild(ctx, S));
    while ((int32_t)S.inflight.size() < S.depth) {
        const int32_t lim = (S.mode == VH_SERVE_SEQUENTIAL) ? 1 : (S.max_batch > 0 ? S.max_batch : 1 << 30);
        std::vector<int32_t> ids = S.pol.pick(lim);
        if (ids.empty()) break;
        VH_TRY(launch(S, ids));
        ++n;
    }
    if (wait && n == 0 && !S.inflight.empty()) VH_TRY(retire(S, true));
    if (n_launched) *n_launched = n;
    return VH_OK;
}

Server* server_of(vh_ctx* ctx) { return ctx ? ctx->srv : nullptr; }

int member_of(vh_ctx* ctx, vh_mesh* m, int32_t* id) {
    Server* S = server_of(ctx);
    if (!S) return fail(VH_ESTATE, "the server is not open");
    if (!m || m->ctx != ctx || m->srv_id < 0 || m->srv_id >= (int32_t)S->mesh.size() || S->mesh[m->srv_id] != m)
        return fail(VH_EINVAL, "mesh is not in this context's server");
    *id = m->srv_id;
    return VH_OK;
}

}  // namespace

int server_check_idle(vh_mesh* m) {
    Server* S = m->ctx ? m->ctx->srv : nullptr;
    if (!S || m->srv_id < 0) return VH_OK;
    if (!S->pol.idle(m->srv_id)) return fail(VH_ESTATE, "mesh has server frames outstanding");
    return VH_OK;
}

void server_destroy(vh_ctx* ctx) {
    Server* S = ctx ? ctx->srv : nullptr;
    if (!S) return;
    (void)drain(*S);
    (void)free_batched(ctx, *S);
    for (vh_mesh* m : S->mesh)
        if (m) m->srv_id = -1;
    for (hipEvent_t e : S->ev_free) (void)hipEventDestroy(e);
    for (auto& B : S->inflight) (void)hipEventDestroy(B.done);
    if (S->ev0) (void)hipEventDestroy(S->ev0);
    if (S->cap) (void)hipStreamDestroy(S->cap);
    if (S->s) (void)hipStreamDestroy(S->s);
    delete S;
    ctx->srv = nullptr;
}

}  // namespace vhrt

using namespace vhrt;

extern "C" {

int vh_serve_open(vh_ctx* ctx, int32_t mode, int32_t max_in_flight, int32_t max_batch) {
    if (!ctx) return fail(VH_EINVAL, "null context");
    if (ctx->srv) return fail(VH_ESTATE, "the server is already open");
    if (mode != VH_SERVE_BATCHED && mode != VH_SERVE_SEQUENTIAL) return fail(VH_EINVAL, "unknown serve mode");
    if (max_in_flight < 1 || max_in_flight > 64) return fail(VH_EINVAL, "max_in_flight must be in 1..64");
    if (max_batch < 0) return fail(VH_EINVAL, "max_batch must be >= 0");
    VH_HIP(hipSetDevice(ctx->device));
    Server* S = new Server();
    S->mode = mode;
    S->depth = max_in_flight;
    S->max_batch = max_batch;
    S->use_graph = ctx->cfg.use_graphs != 0;
    ctx->srv = S;
    auto bail = [&](hipError_t e, const char* what) {
        server_destroy(ctx);
        return fail(VH_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
    };
    hipError_t e = hipStreamCreateWithFlags(&S->s, hipStreamNonBlocking);
    if (e != hipSuccess) return bail(e, "hipStreamCreateWithFlags");
    e = hipEventCreate(&S->ev0);
    if (e != hipSuccess) return bail(e, "hipEventCreate");
    e = hipEventRecord(S->ev0, S->s);
    if (e == hipSuccess) e = hipEventSynchronize(S->ev0);
    if (e != hipSuccess) return bail(e, "clock origin");
    S->t0 = std::chrono::steady_clock::now();
    ctx->peak = ctx->in_use;                 // the HBM peak of this server's lifetime
    return VH_OK;
}

int vh_serve_close(vh_ctx* ctx) {
    Server* S = server_of(ctx);
    if (!S) return fail(VH_ESTATE, "the server is not open");
    VH_HIP(hipSetDevice(ctx->device));
    VH_TRY(drain(*S));
    VH_TRY(apply_releases(ctx, *S));
    server_destroy(ctx);
    return VH_OK;
}

int vh_serve_add(vh_ctx* ctx, vh_mesh* m, int32_t n_subdomains, int32_t refine_steps) {
    Server* S = server_of(ctx);
    if (!S) return fail(VH_ESTATE, "the server is not open");
    if (!m || m->ctx != ctx) return fail(VH_EINVAL, "mesh does not belong to this context");
    if (m->srv_id >= 0) return fail(VH_EINVAL, "mesh is already in the server");
    VH_TRY(set_device(m));
    if (!m->factored && !m->planned) VH_TRY(host_factor(m, n_subdomains, refine_steps));
    if (!m->factored) {
        size_t need = 0;
        VH_TRY(device_need(m, &need));
        if (ctx->budget && need > ctx->budget)
            return fail(VH_ENOMEM, "mesh needs " + std::to_string(need) + " device bytes, more than the budget");
    }
    if (S->pd_iters < 0) {
        S->pd_iters = m->plan.pd_iters;
        S->refine = m->refine;
    } else if (m->plan.pd_iters != S->pd_iters || m->refine != S->refine) {
        return fail(VH_EINVAL, "meshes of one server need equal pd_iters and refine steps");
    }
    // a batched launch gives every workgroup the LDS of the largest subdomain
    // of any garment in it
    const int32_t mn = std::max(S->max_n, std::max(m->plan.max_sub_n, 1));
    const int32_t mb = std::max(S->max_nb, m->plan.max_nb), mc = std::max(S->max_cint, m->plan.max_cint);
    if (S->mode == VH_SERVE_BATCHED) {
        int lds_limit = 0;
        VH_HIP(hipDeviceGetAttribute(&lds_limit, hipDeviceAttributeMaxSharedMemoryPerBlock, ctx->device));
        const size_t lds = std::max(vh::interior_fwd_lds(mn, mc), vh::interior_bwd_lds(mn, mb));
        if (lds > (size_t)lds_limit)
            return fail(VH_EINVAL, "a batched launch with this mesh needs " + std::to_string(lds) +
                                       " bytes of LDS (limit " + std::to_string(lds_limit) +
                                       "); give it or the others more subdomains");
    }
    S->max_n = mn;
    S->max_nb = mb;
    S->max_cint = mc;
    size_t need = 0;
    if (!m->factored) VH_TRY(device_need(m, &need));
    const int32_t id = S->pol.add_garment();
    S->pol.set_need(id, need);
    S->mesh.push_back(m);
    S->release_req.push_back(0);
    S->pos.push_back(-1);
    m->srv_id = id;
    if (m->factored) {
        if (m->ctx->cfg.use_graphs) VH_TRY(ensure_graph(m));
        S->pol.admit(id);
        S->dirty = true;
    }
    return VH_OK;
}

int vh_serve_submit(vh_ctx* ctx, vh_mesh* m, int32_t n_frames, double t_arrival, uint64_t* ticket) {
    int32_t id = -1;
    VH_TRY(member_of(ctx, m, &id));
    if (n_frames < 1) return fail(VH_EINVAL, "n_frames must be >= 1");
    if (!ticket) return fail(VH_EINVAL, "null ticket");
    Server& S = *ctx->srv;
    if (S.release_req[id]) return fail(VH_ESTATE, "mesh is being released");
    const double t = (t_arrival < 0.0) ? host_now(S) : t_arrival;
    *ticket = S.pol.submit(id, n_frames, t);
    return VH_OK;
}

int vh_serve_tick(vh_ctx* ctx, int32_t wait, int32_t* n_launched) {
    Server* S = server_of(ctx);
    if (!S) return fail(VH_ESTATE, "the server is not open");
    VH_HIP(hipSetDevice(ctx->device));
    return tick(ctx, *S, wait != 0, n_launched);
}

int vh_serve_drain(vh_ctx* ctx) {
    Server* S = server_of(ctx);
    if (!S) return fail(VH_ESTATE, "the server is not open");
    VH_HIP(hipSetDevice(ctx->device));
    while (S->pol.any_pending()) {
        int32_t n = 0;
        VH_TRY(tick(ctx, *S, true, &n));
        if (n == 0 && S->inflight.empty() && S->pol.any_pending()) {
            // nothing runs and nothing can: the waiting requests belong to
            // garments that do not fit next to the resident ones
            VH_TRY(apply_releases(ctx, *S));
            VH_TRY(admit(ctx, *S));
            if (S->pol.pick(1).empty())
                return fail(VH_ESTATE, "requests wait for garments that cannot be admitted; release resident meshes");
        }
    }
    VH_TRY(drain(*S));
    return apply_releases(ctx, *S);
}

int vh_serve_release(vh_ctx* ctx, vh_mesh* m) {
    int32_t id = -1;
    VH_TRY(member_of(ctx, m, &id));
    VH_HIP(hipSetDevice(ctx->device));
    Server& S = *ctx->srv;
    if (S.pol.state(id) == vh::ServePolicy::QUEUED && S.pol.idle(id)) {
        S.pol.release(id);                   // never on the device
        S.mesh[id] = nullptr;
        m->srv_id = -1;
        return VH_OK;
    }
    // a queued mesh with requests is still admitted, runs them, then leaves
    S.release_req[id] = 1;
    VH_TRY(retire(S, false));
    return apply_releases(ctx, S);
}

int vh_serve_poll(vh_ctx* ctx, uint64_t ticket, int32_t* done, double* latency_s) {
    Server* S = server_of(ctx);
    if (!S) return fail(VH_ESTATE, "the server is not open");
    if (!done) return fail(VH_EINVAL, "null argument");
    const vh::ServeRequest* r = S->pol.find(ticket);
    if (!r) return fail(VH_EINVAL, "unknown ticket");
    *done = (r->done == r->frames) ? 1 : 0;
    if (latency_s) *latency_s = *done ? r->t_done - r->t_arrival : -1.0;
    return VH_OK;
}

int vh_serve_now(vh_ctx* ctx, double* t) {
    Server* S = server_of(ctx);
    if (!S) return fail(VH_ESTATE, "the server is not open");
    if (!t) return fail(VH_EINVAL, "null argument");
    *t = host_now(*S);
    return VH_OK;
}

int vh_serve_time_kernel(vh_ctx* ctx, int32_t kernel_class, int32_t reps, void* stream) {
    Server* S = server_of(ctx);
    if (!S) return fail(VH_ESTATE, "the server is not open");
    if (S->mode != VH_SERVE_BATCHED) return fail(VH_ESTATE, "kernel timing needs a batched server");
    if (reps < 1) return fail(VH_EINVAL, "reps must be >= 1");
    if (kernel_class != 1 && kernel_class != 2) return fail(VH_EINVAL, "kernel_class must be 1 or 2");
    VH_HIP(hipSetDevice(ctx->device));
    VH_TRY(drain(*S));
    if (S->dirty) VH_TRY(rebuild(ctx, *S));
    if (S->ls.ng == 0) return fail(VH_ESTATE, "no resident mesh");
    std::vector<int32_t> on(S->ls.ng, 0);
    for (int32_t g = 0; g < (int32_t)S->pos.size(); ++g)
        if (S->pos[g] >= 0) on[S->pos[g]] = 1;
    VH_HIP(hipMemcpy(S->ls.active, on.data(), sizeof(int32_t) * S->ls.ng, hipMemcpyHostToDevice));
    hipStream_t s = static_cast<hipStream_t>(stream);
    for (int32_t r = 0; r < reps; ++r) {
        if (kernel_class == 1) VH_HIP(vh::launch_local(S->ls.local, s, false));
        else VH_HIP(vh::launch_residual(S->ls.residual, s));
    }
    return VH_OK;
}

int vh_serve_reset_stats(vh_ctx* ctx) {
    Server* S = server_of(ctx);
    if (!S) return fail(VH_ESTATE, "the server is not open");
    VH_HIP(hipSetDevice(ctx->device));
    VH_TRY(retire(*S, false));
    S->pol.reset_stats();
    S->launches = 0;
    S->garment_frames = 0;
    ctx->peak = ctx->in_use;
    return VH_OK;
}

int vh_serve_get_stats(vh_ctx* ctx, vh_serve_stats* st) {
    Server* S = server_of(ctx);
    if (!S) return fail(VH_ESTATE, "the server is not open");
    if (!st) return fail(VH_EINVAL, "null argument");
    const vh::ServePolicy& P = S->pol;
    st->frames_done = P.frames_done();
    st->requests_done = P.requests_done();
    st->launches = S->launches;
    st->mean_batch = S->launches ? (double)S->garment_frames / (double)S->launches : 0.0;
    st->span_s = P.span();
    st->frames_per_second = st->span_s > 0.0 ? (double)st->frames_done / st->span_s : 0.0;
    st->latency_p50_s = P.percentile(0.50);
    st->latency_p99_s = P.percentile(0.99);
    st->latency_max_s = P.percentile(1.0);
    st->hbm_in_use = ctx->in_use;
    st->hbm_peak = ctx->peak;
    int32_t res = 0, wait = 0;
    for (int32_t g = 0; g < P.n_garments(); ++g) {
        if (P.state(g) == vh::ServePolicy::RESIDENT) ++res;
        if (P.state(g) == vh::ServePolicy::QUEUED) ++wait;
    }
    st->meshes_resident = res;
    st->meshes_waiting = wait;
    return VH_OK;
}

}  // extern "C"
