// Numeric factorization of the interface supernodes on the device: the dense
// part of the prefactor (the interface Schur complement of Sec. 7.2 and the
// blocks its solve applies).  Per interface supernode, in the plan's order
// (children before parents):
//   * the frontal matrix F (f = n + m, column-major, lower triangle) gathers
//     the global matrix's entries of the supernode's columns and the update
//     matrices of its children (interior children's from the host, interface
//     children's from their fronts on the device);
//   * F11 = L11 L11^T (potrf), L21 = F21 L11^-T (trsm), F22 -= L21 L21^T (syrk:
//     the update matrix passed to the parent), Ti = L11^-1 (trtri),
//     W_B = L21 Ti (trmm); a root's A = Ti^T Ti (syrk);
//   * Ti, W_B (or A) are written into the device factor in the layouts the
//     interface phases read (the host's packing of the same blocks).
// The dense steps are rocSOLVER / rocBLAS FP64 (matrix cores on gfx950), with
// atomics disallowed so that every factorization of the same matrix is the same.
#include <hip/hip_runtime.h>
#include <rocblas/rocblas.h>
#include <rocsolver/rocsolver.h>

#include <algorithm>
#include <cmath>
#include <string>
#include <vector>

#include "runtime.h"

namespace vh {
namespace {

constexpr int TB = 16;   // 16 x 16 thread tiles of the assembly and packing kernels

// F[dest[i]] += kval[src[i]]: the global matrix's lower entries of the
// supernode's columns (each destination once)
__global__ __launch_bounds__(256) void k_front_matrix(double* __restrict__ F, const int64_t* __restrict__ dest,
                                                      const int32_t* __restrict__ src, int32_t cnt,
                                                      const double* __restrict__ kval) {
    const int32_t i = blockIdx.x * 256 + threadIdx.x;
    if (i < cnt) F[dest[i]] += kval[src[i]];
}

// Extend-add of a child's update matrix U (lower part: U(a, b) = U[b * ldu + a]
// for a >= b) into F at the child's rows' positions map[0..mc) (increasing, so
// the lower triangle lands in F's lower triangle)
__global__ __launch_bounds__(TB * TB) void k_front_add(double* __restrict__ F, int64_t ldf,
                                                       const double* __restrict__ U, int64_t ldu,
                                                       const int32_t* __restrict__ map, int32_t mc) {
    const int32_t a = blockIdx.x * TB + threadIdx.x, b = blockIdx.y * TB + threadIdx.y;
    if (a >= mc || b >= mc || a < b) return;
    F[(int64_t)map[b] * ldf + map[a]] += U[(int64_t)b * ldu + a];
}

// Ti (n x n, column-major lower) and W_B (m x n, column-major) into the
// forward block (rows of [Ti; W_B], the triangle row-major) and the backward
// block (per column k: Ti[k..n)[k], then -W_B[.][k]) of a supernode
__global__ __launch_bounds__(TB * TB) void k_pack_blocks(double* __restrict__ vals, int64_t wf_off, int64_t wb_off,
                                                         const double* __restrict__ Ti,
                                                         const double* __restrict__ WB, int32_t n, int32_t m) {
    const int32_t a = blockIdx.x * TB + threadIdx.x, r = blockIdx.y * TB + threadIdx.y;
    if (a >= n || r >= n + m) return;
    const int64_t col = wb_off + (int64_t)a * (n + m) - (int64_t)a * (a - 1) / 2;   // column a's backward run
    if (r < n) {
        if (a > r) return;
        const double t = Ti[(int64_t)a * n + r];
        vals[wf_off + (int64_t)r * (r + 1) / 2 + a] = t;
        vals[col + (r - a)] = t;
    } else {
        const int32_t p = r - n;
        const double w = WB[(int64_t)a * m + p];
        vals[wf_off + (int64_t)n * (n + 1) / 2 + (int64_t)p * n + a] = w;
        vals[col + (n - a) + p] = -w;
    }
}

// A root's symmetric A (column-major lower) as a full row-major n x n block
__global__ __launch_bounds__(TB * TB) void k_pack_root(double* __restrict__ vals, int64_t off,
                                                       const double* __restrict__ A, int32_t n) {
    const int32_t j = blockIdx.x * TB + threadIdx.x, i = blockIdx.y * TB + threadIdx.y;
    if (i >= n || j >= n) return;
    vals[off + (int64_t)i * n + j] = (i >= j) ? A[(int64_t)j * n + i] : A[(int64_t)i * n + j];
}

}  // namespace
}  // namespace vh

namespace vhrt {

namespace {

// device buffers of one factorization, freed on every exit
struct Buffers {
    std::vector<void*> p;
    ~Buffers() {
        for (void* q : p) (void)hipFree(q);
    }
    template <class T>
    int get(T** out, size_t count) {
        void* q = nullptr;
        const hipError_t e = hipMalloc(&q, std::max<size_t>(count, 1) * sizeof(T));
        if (e != hipSuccess) return fail(VH_ENOMEM, std::string("hipMalloc (interface factorization): ") +
                                                        hipGetErrorString(e));
        p.push_back(q);
        *out = static_cast<T*>(q);
        return VH_OK;
    }
};

int blas_ok(rocblas_status st, const char* what) {
    if (st == rocblas_status_success) return VH_OK;
    return fail(VH_EDEVICE, std::string(what) + ": " + rocblas_status_to_string(st));
}

// one child's extend-add: its update matrix (a device front or an upload)
struct ChildAdd {
    int32_t child;
    int64_t map_off;
    int32_t mc;
    int64_t up_off;   // offset of an uploaded interior update matrix, -1 for a device front
};

}  // namespace

int blas_handle(vh_ctx* ctx, void** out) {
    if (!ctx->blas) {
        rocblas_handle h = nullptr;
        VH_TRY(blas_ok(rocblas_create_handle(&h), "rocblas_create_handle"));
        (void)rocblas_set_atomics_mode(h, rocblas_atomics_not_allowed);
        ctx->blas = h;
    }
    *out = ctx->blas;
    return VH_OK;
}

void blas_destroy(vh_ctx* ctx) {
    if (ctx->blas) (void)rocblas_destroy_handle(static_cast<rocblas_handle>(ctx->blas));
    ctx->blas = nullptr;
}

int device_interface_factor(vh_mesh* m) {
    vh::Plan& P = m->plan;
    const vh::DevMesh& d = m->dm;
    const std::vector<vh::Supernode>& SN = P.sn;
    const int32_t nsn = (int32_t)SN.size(), nf = P.n_free;
    std::vector<int32_t> order;
    for (int32_t t = 0; t < nsn; ++t)
        if (SN[t].sub < 0) order.push_back(t);
    if (order.empty()) {
        P.dvals_ready = true;
        P.iface_child_upd.clear();
        return VH_OK;
    }
    void* hv = nullptr;
    VH_TRY(blas_handle(m->ctx, &hv));
    rocblas_handle h = static_cast<rocblas_handle>(hv);
    VH_TRY(blas_ok(rocblas_set_stream(h, nullptr), "rocblas_set_stream"));

    // host side: front offsets, the matrix entries of each front, children's maps
    std::vector<int64_t> front(nsn, -1), kbeg(nsn, 0);
    std::vector<int64_t> kdest;
    std::vector<int32_t> ksrc, maps;
    std::vector<double> ups;
    std::vector<std::vector<ChildAdd>> adds(nsn);
    std::vector<int32_t> pos(nf, 0);
    int64_t arena = 0, tsz = 1, wsz = 1;
    for (int32_t t : order) {
        const vh::Supernode& s = SN[t];
        const int32_t n = s.n, mr = (int32_t)s.rows.size(), f = n + mr;
        front[t] = arena;
        arena += (int64_t)f * f;
        tsz = std::max<int64_t>(tsz, (int64_t)n * n);
        wsz = std::max<int64_t>(wsz, mr > 0 ? (int64_t)mr * n : (int64_t)n * n);
        for (int32_t a = 0; a < n; ++a) pos[s.col0 + a] = a;
        for (int32_t b = 0; b < mr; ++b) pos[s.rows[b]] = n + b;
        kbeg[t] = (int64_t)kdest.size();
        for (int32_t a = 0; a < n; ++a) {
            const int32_t j = s.col0 + a;
            for (int32_t k = P.K_ptr[j]; k < P.K_ptr[j + 1]; ++k) {
                const int32_t i = P.K_col[k];
                if (i < j) continue;
                kdest.push_back((int64_t)a * f + pos[i]);
                ksrc.push_back(k);
            }
        }
        for (int32_t c : s.children) {
            const vh::Supernode& cs = SN[c];
            const int32_t mc = (int32_t)cs.rows.size();
            if (mc == 0) continue;
            ChildAdd ca{c, (int64_t)maps.size(), mc, -1};
            for (int32_t b = 0; b < mc; ++b) maps.push_back(pos[cs.rows[b]]);
            if (cs.sub >= 0) {
                const std::vector<double>& U = P.iface_child_upd.at(c);
                if ((int64_t)U.size() != (int64_t)mc * mc) return fail(VH_ESTATE, "interior update matrix missing");
                ca.up_off = (int64_t)ups.size();
                ups.insert(ups.end(), U.begin(), U.end());
            }
            adds[t].push_back(ca);
        }
    }

    Buffers B;
    double *F = nullptr, *T = nullptr, *W = nullptr, *U = nullptr;
    int64_t* kd = nullptr;
    int32_t *ks = nullptr, *mp = nullptr;
    rocblas_int* info = nullptr;
    VH_TRY(B.get(&F, (size_t)arena));
    VH_TRY(B.get(&T, (size_t)tsz));
    VH_TRY(B.get(&W, (size_t)wsz));
    VH_TRY(B.get(&U, ups.size()));
    VH_TRY(B.get(&kd, kdest.size()));
    VH_TRY(B.get(&ks, ksrc.size()));
    VH_TRY(B.get(&mp, maps.size()));
    VH_TRY(B.get(&info, 2 * order.size()));
    VH_HIP(hipMemset(F, 0, (size_t)arena * sizeof(double)));
    VH_HIP(hipMemset(info, 0, 2 * order.size() * sizeof(rocblas_int)));
    if (!ups.empty()) VH_HIP(hipMemcpy(U, ups.data(), ups.size() * sizeof(double), hipMemcpyHostToDevice));
    if (!kdest.empty()) {
        VH_HIP(hipMemcpy(kd, kdest.data(), kdest.size() * sizeof(int64_t), hipMemcpyHostToDevice));
        VH_HIP(hipMemcpy(ks, ksrc.data(), ksrc.size() * sizeof(int32_t), hipMemcpyHostToDevice));
    }
    if (!maps.empty()) VH_HIP(hipMemcpy(mp, maps.data(), maps.size() * sizeof(int32_t), hipMemcpyHostToDevice));

    const double one = 1.0, minus_one = -1.0, zero = 0.0;
    for (size_t q = 0; q < order.size(); ++q) {
        const int32_t t = order[q];
        const vh::Supernode& s = SN[t];
        const int32_t n = s.n, mr = (int32_t)s.rows.size(), f = n + mr;
        double* Ft = F + front[t];
        // the matrix entries of this front: [kbeg[t], next front's kbeg)
        const int64_t k0 = kbeg[t];
        const int64_t k1 = (q + 1 < order.size()) ? kbeg[order[q + 1]] : (int64_t)kdest.size();
        const int32_t kc = (int32_t)(k1 - k0);
        if (kc > 0)
            hipLaunchKernelGGL(vh::k_front_matrix, dim3((kc + 255) / 256), dim3(256), 0, nullptr, Ft, kd + k0,
                               ks + k0, kc, d.K_val);
        for (const ChildAdd& ca : adds[t]) {
            const vh::Supernode& cs = SN[ca.child];
            const double* Uc;
            int64_t ldu;
            if (ca.up_off >= 0) {
                Uc = U + ca.up_off;
                ldu = ca.mc;
            } else {
                const int64_t fc = cs.n + (int64_t)cs.rows.size();
                Uc = F + front[ca.child] + (int64_t)cs.n * fc + cs.n;
                ldu = fc;
            }
            const dim3 g((ca.mc + vh::TB - 1) / vh::TB, (ca.mc + vh::TB - 1) / vh::TB);
            hipLaunchKernelGGL(vh::k_front_add, g, dim3(vh::TB, vh::TB), 0, nullptr, Ft, (int64_t)f, Uc, ldu,
                               mp + ca.map_off, ca.mc);
        }
        VH_HIP(hipGetLastError());
        VH_TRY(blas_ok(rocsolver_dpotrf(h, rocblas_fill_lower, n, Ft, f, info + 2 * q), "rocsolver_dpotrf"));
        if (mr > 0) {
            VH_TRY(blas_ok(rocblas_dtrsm(h, rocblas_side_right, rocblas_fill_lower, rocblas_operation_transpose,
                                         rocblas_diagonal_non_unit, mr, n, &one, Ft, f, Ft + n, f),
                           "rocblas_dtrsm"));
            VH_TRY(blas_ok(rocblas_dsyrk(h, rocblas_fill_lower, rocblas_operation_none, mr, n, &minus_one, Ft + n, f,
                                         &one, Ft + (int64_t)n * f + n, f),
                           "rocblas_dsyrk"));
        }
        VH_HIP(hipMemcpy2DAsync(T, (size_t)n * sizeof(double), Ft, (size_t)f * sizeof(double),
                                (size_t)n * sizeof(double), (size_t)n, hipMemcpyDeviceToDevice, nullptr));
        VH_TRY(blas_ok(rocsolver_dtrtri(h, rocblas_fill_lower, rocblas_diagonal_non_unit, n, T, n, info + 2 * q + 1),
                       "rocsolver_dtrtri"));
        if (mr > 0) {
            VH_TRY(blas_ok(rocblas_dtrmm(h, rocblas_side_right, rocblas_fill_lower, rocblas_operation_none,
                                         rocblas_diagonal_non_unit, mr, n, &one, T, n, Ft + n, f, W, mr),
                           "rocblas_dtrmm"));
            const dim3 g((n + vh::TB - 1) / vh::TB, (n + mr + vh::TB - 1) / vh::TB);
            hipLaunchKernelGGL(vh::k_pack_blocks, g, dim3(vh::TB, vh::TB), 0, nullptr, d.dvals, s.wf_off, s.wb_off, T,
                               W, n, mr);
        } else {
            VH_TRY(blas_ok(rocblas_dsyrk(h, rocblas_fill_lower, rocblas_operation_transpose, n, n, &one, T, n, &zero,
                                         W, n),
                           "rocblas_dsyrk"));
            const dim3 g((n + vh::TB - 1) / vh::TB, (n + vh::TB - 1) / vh::TB);
            hipLaunchKernelGGL(vh::k_pack_root, g, dim3(vh::TB, vh::TB), 0, nullptr, d.dvals, s.wf_off, W, n);
        }
        VH_HIP(hipGetLastError());
    }
    VH_HIP(hipDeviceSynchronize());
    std::vector<rocblas_int> hinfo(2 * order.size());
    VH_HIP(hipMemcpy(hinfo.data(), info, hinfo.size() * sizeof(rocblas_int), hipMemcpyDeviceToHost));
    for (rocblas_int v : hinfo)
        if (v != 0) return fail(VH_ENOTSPD, "non-positive pivot in the interface factor");
    // the host plan keeps the same values (a later upload, e.g. by the server)
    VH_HIP(hipMemcpy(P.dvals.data(), d.dvals, P.dvals.size() * sizeof(double), hipMemcpyDeviceToHost));
    for (double v : P.dvals)
        if (!std::isfinite(v)) return fail(VH_ENOTSPD, "non-finite value in the interface factor");
    P.dvals_ready = true;
    P.iface_child_upd.clear();
    return VH_OK;
}

}  // namespace vhrt
