// Host-side runtime shared by the mesh entry points (api.hip) and the step
// server (serve.hip): the handle structures, device-memory accounting, the
// launch set of one frame and the helpers that enqueue it.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <utility>
#include <vector>

#include "../../include/vhpd.h"
#include "kernels.h"
#include "plan.h"

#define VH_HIP(call)                                                                         \
    do {                                                                                     \
        hipError_t e_ = (call);                                                              \
        if (e_ != hipSuccess)                                                                \
            return ::vhrt::fail(VH_EDEVICE, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

#define VH_TRY(expr)                  \
    do {                              \
        int rc_ = (expr);             \
        if (rc_ != VH_OK) return rc_; \
    } while (0)

namespace vhrt {

// records msg as the calling thread's last error and returns code
int fail(int code, const std::string& msg);

struct CoarseLaunch {
    vh::LaunchRef ref;
    int32_t kind = 0, group = 16;
};

// The launches of one frame over a set of garments (one mesh, or a batch).
struct LaunchSet {
    vh::DevMesh* G = nullptr;       // device [ng]
    int32_t* tables = nullptr;      // device launch tables
    int32_t* active = nullptr;      // device [ng]
    int32_t ng = 0;
    vh::LaunchRef predict, local, residual, ifwd, ibwd, refine, velocity;
    std::vector<CoarseLaunch> cfwd, cbwd;
    size_t lds_fwd = 0, lds_bwd = 0, lds_cms = 0;
    int32_t pd_iters = 10, refine_steps = 0;
    int32_t cms_modes = 0, cms_sweeps = 0;   // inexact CMS solve when cms_modes > 0
    size_t bytes = 0;
};

struct Server;

}  // namespace vhrt

struct vh_ctx {
    int device = 0;
    vh_config cfg{1, 96, 384, 1, 3000, 0, 10, 64};
    void* scratch = nullptr;        // device address of the step scratch array (vh_mesh_step_noalloc)
    void* blas = nullptr;           // rocBLAS handle of the interface factorization (created on first use)
    size_t budget = 0;
    size_t in_use = 0, peak = 0;
    std::vector<vh_mesh*> meshes;
    vhrt::Server* srv = nullptr;
};

struct vh_mesh {
    vh_ctx* ctx = nullptr;
    int32_t nv = 0, nt = 0;
    std::vector<double> X;
    std::vector<int32_t> tets;
    bool has_params = false;
    bool planned = false;           // host factorization done (plan valid)
    bool factored = false;          // plan resident on the device
    std::vector<double> gs, gv, mass;
    std::vector<uint8_t> pinned;
    double g[3] = {0, 0, 0};
    double dt = 0;
    int32_t iters = 10;
    vh::Plan plan;
    vh::CmsPlan cms;                // inexact CMS data (cms.modes > 0 when selected)
    vh::DevMesh dm;
    std::vector<void*> allocs;
    size_t bytes = 0;
    bool dry = false;               // dalloc/upload only count bytes
    size_t dry_bytes = 0;
    vhrt::LaunchSet ls;             // this mesh's own frame (one garment)
    int32_t refine = 0;
    std::vector<double> stage;      // host staging, nv*3
    // last state kept on the host when the mesh left the device (server release)
    bool has_saved = false;
    std::vector<double> saved_x, saved_v;
    int32_t srv_id = -1;            // garment id in the context's server, -1 if none
    // optional per-kernel-class timing with HIP events on the step's stream
    uint32_t prof_mask = 0;
    std::vector<hipEvent_t> ev_pool;
    size_t ev_used = 0;
    std::vector<std::pair<size_t, int>> ev_pairs;   // start event index, class
    // one frame captured as a HIP graph (replayed per frame on the caller's
    // stream while the context's use_graphs is set)
    hipStream_t cap = nullptr;
    hipGraphExec_t gexec = nullptr;
    // adjoint: checkpoints of the last vh_mesh_adjoint_forward (device, owned)
    int32_t adj_frames = 0, adj_every = 0;
    double* adj_ckpt = nullptr;     // [n_ckpt][2][nv][3] (x, v), internal order
    size_t adj_ckpt_bytes = 0;
    // embedded points (Eq. m2y): host definition, and device records built
    // from it while the mesh is resident (freed with the device data)
    std::vector<int32_t> emb_tet;   // user element per point
    std::vector<double> emb_X;      // rest positions [n][3]
    float4* emb_rec = nullptr;      // 2 float4 per point
    double* emb_out = nullptr;      // [n][3] device staging for host reads
    size_t emb_bytes = 0;
};

namespace vhrt {

int set_device(vh_mesh* m);
void free_embedding_device(vh_mesh* m);
// host FP64 factorization into m->plan (no device memory)
int host_factor(vh_mesh* m, int32_t n_subdomains, int32_t refine_steps);
// device bytes the upload of m->plan will take (budgeted allocations)
int device_need(vh_mesh* m, size_t* bytes);
// uploads m->plan, sets the state to rest, builds the mesh's own launch set
int upload_device(vh_mesh* m);
// the interface supernodes' numeric factorization on the device (rocSOLVER /
// rocBLAS FP64) into the resident factor, copied back into the host plan
int device_interface_factor(vh_mesh* m);
int blas_handle(vh_ctx* ctx, void** out);
void blas_destroy(vh_ctx* ctx);
// frees every device buffer of the mesh (state included)
void free_device(vh_mesh* m);
// frees the adjoint checkpoints of the mesh
void free_adjoint(vh_mesh* m);
void charge(vh_ctx* ctx, size_t bytes);
void uncharge(vh_ctx* ctx, size_t bytes);

// Launch tables of one frame over `members` (device-resident, equal pd_iters
// and refine steps).  Device memory is counted in ctx; with check_budget the
// call fails with VH_ENOMEM when it would exceed the budget.
int build_launch_set(vh_ctx* ctx, const std::vector<vh_mesh*>& members, LaunchSet& L,
                     bool check_budget);
void free_launch_set(vh_ctx* ctx, LaunchSet& L);

// A launch of L's tables with the garment records at G instead (G null: L's own).
inline vh::LaunchRef with_record(const vh::LaunchRef& r, const vh::DevMesh* G) {
    vh::LaunchRef o = r;
    if (G) o.G = G;
    return o;
}

// One frame over the launch set on s; prof (may be null) receives per-class
// timing; G (may be null) replaces the launch set's device records.
int frame_direct(vh_mesh* prof, const LaunchSet& L, hipStream_t s, const vh::DevMesh* G = nullptr);
// Capture frame_direct(L) on `cap` into an executable graph.
int capture_frame(const LaunchSet& L, hipStream_t* cap, hipGraphExec_t* out);
// the mesh's own frame graph, captured on first use
int ensure_graph(vh_mesh* m);

// internal device rows -> user-ordered host array [nv][3] (rows >= n given are 0)
int get_user(vh_mesh* m, const double* dev_int, double* host, int32_t rows, hipStream_t s);
// user-ordered host [nv][3] -> internal device rows (pinned rows: X if positions, else 0); synchronises s
int put_user(vh_mesh* m, const double* host, double* dev_int, bool positions, hipStream_t s);

// d = K^{-1} r on the mesh's device vectors (r -> delta; apply: x += d);
// resid: r is first formed as the PD residual from the local step's partials
int solve(vh_mesh* m, const LaunchSet& L, hipStream_t s, bool apply, bool keep_delta,
          const vh::DevMesh* G = nullptr, bool resid = false);
// one local/global iteration (local step, residual, solve with refinement, x += d)
int pd_iteration(vh_mesh* m, const LaunchSet& L, hipStream_t s, const vh::DevMesh* G = nullptr);

// ctx->scratch = the device address of the step scratch array on the current
// device (hipGetSymbolAddress); called once per context, its device current
int noalloc_init(vh_ctx* ctx);
// VH_ESTATE unless the mesh is prefactored; check_solo: and not driven by a
// server; check_quiet: and no server frames of it pending
int check_ready(vh_mesh* m);
int check_solo(vh_mesh* m);
int check_quiet(vh_mesh* m);

// server teardown (drains its launches); called by vh_ctx_destroy
void server_destroy(vh_ctx* ctx);
// VH_ESTATE if the mesh belongs to a server and has frames submitted or running
int server_check_idle(vh_mesh* m);

}  // namespace vhrt
