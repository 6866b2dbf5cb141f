// Device kernels of the PD step (gfx950).  Launch helpers are declared here
// and defined in kernels.hip; every launch takes the caller's stream.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "plan.h"

namespace vh {

// Device-resident copy of a Plan plus the state of one garment.
struct DevMesh {
    int32_t nv = 0, nt = 0, n_free = 0, n_int = 0, n_gamma = 0, D = 1;
    int32_t max_sub_n = 0;
    double dt = 0, g[3] = {0, 0, 0};
    // state, internal order, AoS xyz
    double *x = nullptr, *v = nullptr, *xprev = nullptr, *y = nullptr, *X = nullptr;
    double* mass = nullptr;
    int32_t* perm = nullptr;        // internal vertex -> user vertex
    float4* u = nullptr;            // float(x - X), w unused
    // elements
    float4* trec = nullptr;         // [nt][4]: ids, Dm^{-1}, V gs, V gv, V
    uint2* lpos = nullptr;          // [nt]: 4 x uint16 LDS positions of the corner forces
    int32_t *blk_part = nullptr, *part_pack = nullptr;
    float4* part = nullptr;         // per (block, vertex) partial force sums
    int32_t *vpart_ptr = nullptr, *vpart = nullptr;
    // solver
    double* r = nullptr;            // [n_free][3] residual
    float* zf = nullptr;            // [n_int][3] interior forward result
    double *rg = nullptr, *zg = nullptr, *dg = nullptr;   // [n_gamma][3] interface work
    double* delta = nullptr;        // [n_free][3] last correction
    int32_t* sub_off = nullptr;
    Chunk* chunks = nullptr;
    int32_t *sub_fwd_ch = nullptr, *sub_bwd_ch = nullptr;
    float* ivals = nullptr;
    int32_t *bnd = nullptr, *bnd_off = nullptr;
    int32_t max_nb = 0, max_cint = 0;
    int32_t desc_table = 64;        // chunk descriptors held in the interior kernels' LDS table (1..64)
    double* dvals = nullptr;
    CTask* ctasks = nullptr;
    int32_t *cslots = nullptr, *cgidx = nullptr;
    float* cgf = nullptr;           // [n_cgf][3]
    double* cgd = nullptr;          // [n_cgd][3]
    int32_t *K_ptr = nullptr, *K_col = nullptr;
    double* K_val = nullptr;
    uint32_t* flags = nullptr;      // [0] non-finite value seen in the state
    // projection regime counters of the local step (element evaluations):
    // [0] clamped, [1] inverted, [2] det F >= 2, [3] mixed-branch point taken,
    // [4] no + branch root
    unsigned long long* regime = nullptr;
    // inexact CMS solve of Sec. 7.2 (cms_modes > 0): interior eigenmodes
    // (column-major per subdomain at cms_phi_off[d]), their inverse
    // eigenvalues [D][cms_modes], boundary modes Psi_d (column-major per
    // subdomain at cms_psi_off[d], one column per Plan::bnd row), the inverse
    // diagonal of K and the Chebyshev weights of the Jacobi sweeps, and two
    // sweep buffers [n_free][3] (the first is delta)
    int32_t cms_modes = 0, cms_sweeps = 0;
    const float *cms_phi = nullptr, *cms_psi = nullptr, *cms_ilam = nullptr;
    const int64_t *cms_phi_off = nullptr, *cms_psi_off = nullptr;
    const double *cms_invd = nullptr, *cms_omega = nullptr;
    double *cms_b1 = nullptr, *cms_b2 = nullptr;
    double* cms_q = nullptr;        // [D][cms_modes][3] Lambda^{-1} Phi^T b per subdomain
    // debug outputs of the local step (allocated on demand)
    float *dbg_T = nullptr, *dbg_sig = nullptr, *dbg_s = nullptr;
    // the element-colouring cross-check of the scatter (allocated on demand)
    int32_t* dbg_col = nullptr;     // [nt] tets grouped by colour
    float* dbg_b = nullptr;         // [n_free][3] FP32 force sums
};

// One launch over one or more garments: G is a device array of DevMesh, L the
// launch table (device, 16-byte aligned) of one {garment index into G, block
// index within the garment, x0, x1} entry per block, active a device array of
// per-garment flags, nblocks the number of blocks.
struct LaunchRef {
    const DevMesh* G = nullptr;
    const int32_t* L = nullptr;
    const int32_t* active = nullptr;
    int32_t nblocks = 0;
};

// LDS bytes of the interior kernels (two chunk buffers + subdomain vectors)
size_t interior_fwd_lds(int32_t max_n, int32_t max_cint);
size_t interior_bwd_lds(int32_t max_n, int32_t max_nb);
// allow the interior kernels to use up to `bytes` of LDS per workgroup
hipError_t interior_set_lds_limit(size_t bytes);
// capacity of one interior LDS chunk in 32-bit words
int32_t interior_chunk_words();
// blocks per garment of each launch kind
int32_t blocks_vertices(int32_t n);
int32_t blocks_tets(int32_t nt);
int32_t coarse_blocks(int32_t ntasks, int32_t group);

hipError_t launch_predictor(const LaunchRef& r, hipStream_t s);
hipError_t launch_local(const LaunchRef& r, hipStream_t s, bool debug);
// one colour of the element-colouring scatter: the count tets list[0..count)
// (no two share a free vertex) add their corner forces, formed from the debug
// stress dbg_T, into dbg_b
hipError_t launch_scatter_colour(const DevMesh& d, const int32_t* list, int32_t count, hipStream_t s);
hipError_t launch_residual(const LaunchRef& r, hipStream_t s);
// resid: compute the PD residual r first (as launch_residual does) instead of
// reading it
hipError_t launch_interior_fwd(const LaunchRef& r, size_t lds, hipStream_t s, bool resid);
hipError_t launch_coarse(const LaunchRef& r, int32_t kind, int32_t group, hipStream_t s);
hipError_t launch_interior_bwd(const LaunchRef& r, size_t lds, hipStream_t s, bool apply, bool keep_delta);
hipError_t launch_refine_residual(const LaunchRef& r, hipStream_t s);
// inexact CMS solve (after the interior forward and interface solves):
// interior rows from the modes (one block per subdomain; table of ibwd),
// interface rows from the interface solution, Chebyshev-weighted Jacobi sweep
// k, and the final correction to delta (with apply: x += d) (tables over the
// free rows, like refine)
size_t cms_back_lds(int32_t max_n, int32_t max_nb, int32_t modes);
hipError_t launch_cms_back(const LaunchRef& r, size_t lds, int32_t modes, hipStream_t s);
hipError_t launch_cms_iface(const LaunchRef& r, hipStream_t s);
hipError_t launch_cms_sweep(const LaunchRef& r, int32_t k, hipStream_t s);
hipError_t launch_cms_apply(const LaunchRef& r, int32_t sweeps, bool apply, hipStream_t s);
hipError_t launch_velocity(const LaunchRef& r, hipStream_t s);
// embedded points: out[n][3] (internal record order) from the internal state x
hipError_t launch_embed(const float4* rec, const double* x, int32_t n, double* out, hipStream_t s);

}  // namespace vh

namespace vh {
// dst_user[perm[i]] = src_int[i] (3 doubles per vertex), i < nv
hipError_t launch_to_user(int32_t nv, const int32_t* perm, const double* src_int, double* dst_user,
                          hipStream_t s);
// dst_int[i] = i < n_free ? src_user[perm[i]] : fixed (X for positions, 0 for velocities)
hipError_t launch_from_user(int32_t nv, int32_t n_free, const int32_t* perm, const double* src_user,
                            const double* X_or_null, double* dst_int, hipStream_t s);
// u = float(x - X)
hipError_t launch_refresh_u(const DevMesh& m, hipStream_t s);
// discrete adjoint of one PD iteration (one garment; dev_mesh: its device DevMesh):
// gbar += gamma_s term, partials of the J_P [G lambda] corner forces
hipError_t launch_adj_local(const DevMesh* dev_mesh, int32_t nt, const double* xk, const double* xk1,
                            const double* lam, double* gbar, hipStream_t s);
// xbar = sum of partials, ybar += M lambda / dt^2 (free rows)
hipError_t launch_adj_gather(const DevMesh* dev_mesh, int32_t n_free, const double* lam, double* xbar,
                             double* ybar, hipStream_t s);
// adjoint Gauss-Newton (one garment): partials of B d (gathered by
// launch_adj_gather), out = K v - geo on the free rows, FP64 vector helpers
// (partial dot products: gn_dot_blocks() values, summed by the caller)
hipError_t launch_gn_bd(const DevMesh* dev_mesh, int32_t nt, const double* x, const double* dgam, hipStream_t s);
hipError_t launch_gn_av(const DevMesh* dev_mesh, int32_t n_free, const double* v, const double* geo, double* out,
                        hipStream_t s);
hipError_t launch_gn_axpy(int32_t n, double a, const double* x, double* y, hipStream_t s);
hipError_t launch_gn_xpby(int32_t n, const double* x, double b, double* y, hipStream_t s);
int32_t gn_dot_blocks();
hipError_t launch_gn_dot(int32_t n, const double* x, const double* y, double* part, hipStream_t s);
// frame boundaries of the reverse sweep over n3 = 3 n_free values
hipError_t launch_adj_frame(int32_t n3, double dt, bool begin, double* xbar, double* vbar, double* xk, double* xn,
                            double* ybar, hipStream_t s);
}  // namespace vh
