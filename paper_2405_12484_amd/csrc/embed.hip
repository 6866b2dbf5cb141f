// Points embedded in the tetrahedral mesh (Eq. m2y): the positions of yarn
// points driven by the simulated mesh, phi(x) = N x, with N the linear shape
// functions of each point's tet evaluated at the point's rest position.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "runtime.h"

namespace vhrt {

void free_embedding_device(vh_mesh* m) {
    if (m->emb_rec) (void)hipFree(m->emb_rec);
    if (m->emb_out) (void)hipFree(m->emb_out);
    if (m->ctx && m->emb_bytes) uncharge(m->ctx, m->emb_bytes);
    m->emb_rec = nullptr;
    m->emb_out = nullptr;
    m->emb_bytes = 0;
}

namespace {

// Device records of the mesh's embedded points, built on first use while the
// mesh is resident: the shape-function values N_1..3 = Dm^{-1} (X^Y - X_0)
// (Dm = [X_1 - X_0, X_2 - X_0, X_3 - X_0]) in FP64, stored as FP32 with the
// tet's internal vertex ids.
int ensure_embedding(vh_mesh* m) {
    const size_t n = m->emb_tet.size();
    if (n == 0 || m->emb_rec) return VH_OK;
    const vh::Plan& P = m->plan;
    std::vector<float> rec(8 * n);
    for (size_t i = 0; i < n; ++i) {
        const int32_t* t = &m->tets[4 * (size_t)m->emb_tet[i]];
        const double* X0 = &m->X[3 * (size_t)t[0]];
        double D[3][3];   // columns: edges from vertex 0
        for (int a = 0; a < 3; ++a)
            for (int c = 0; c < 3; ++c) D[c][a] = m->X[3 * (size_t)t[a + 1] + c] - X0[c];
        const double det = D[0][0] * (D[1][1] * D[2][2] - D[1][2] * D[2][1]) -
                           D[0][1] * (D[1][0] * D[2][2] - D[1][2] * D[2][0]) +
                           D[0][2] * (D[1][0] * D[2][1] - D[1][1] * D[2][0]);
        double inv[3][3];
        inv[0][0] = (D[1][1] * D[2][2] - D[1][2] * D[2][1]) / det;
        inv[0][1] = (D[0][2] * D[2][1] - D[0][1] * D[2][2]) / det;
        inv[0][2] = (D[0][1] * D[1][2] - D[0][2] * D[1][1]) / det;
        inv[1][0] = (D[1][2] * D[2][0] - D[1][0] * D[2][2]) / det;
        inv[1][1] = (D[0][0] * D[2][2] - D[0][2] * D[2][0]) / det;
        inv[1][2] = (D[0][2] * D[1][0] - D[0][0] * D[1][2]) / det;
        inv[2][0] = (D[1][0] * D[2][1] - D[1][1] * D[2][0]) / det;
        inv[2][1] = (D[0][1] * D[2][0] - D[0][0] * D[2][1]) / det;
        inv[2][2] = (D[0][0] * D[1][1] - D[0][1] * D[1][0]) / det;
        const double d[3] = {m->emb_X[3 * i] - X0[0], m->emb_X[3 * i + 1] - X0[1], m->emb_X[3 * i + 2] - X0[2]};
        float* r = &rec[8 * i];
        for (int a = 0; a < 4; ++a) {
            const int32_t v = P.iperm[t[a]];
            std::memcpy(&r[a], &v, 4);
        }
        for (int a = 0; a < 3; ++a) r[4 + a] = (float)(inv[a][0] * d[0] + inv[a][1] * d[1] + inv[a][2] * d[2]);
        r[7] = 0.0f;
    }
    const size_t rb = rec.size() * sizeof(float), ob = 3 * n * sizeof(double);
    if (m->ctx->budget && m->ctx->in_use + rb + ob > m->ctx->budget)
        return fail(VH_ENOMEM, "HBM budget exceeded (embedded points)");
    VH_HIP(hipMalloc(reinterpret_cast<void**>(&m->emb_rec), rb));
    hipError_t e = hipMalloc(reinterpret_cast<void**>(&m->emb_out), ob);
    if (e != hipSuccess) {
        (void)hipFree(m->emb_rec);
        m->emb_rec = nullptr;
        return fail(VH_ENOMEM, std::string("hipMalloc: ") + hipGetErrorString(e));
    }
    m->emb_bytes = rb + ob;
    charge(m->ctx, m->emb_bytes);
    VH_HIP(hipMemcpy(m->emb_rec, rec.data(), rb, hipMemcpyHostToDevice));
    return VH_OK;
}

}  // namespace
}  // namespace vhrt

using namespace vhrt;

extern "C" {

int vh_mesh_set_embedding(vh_mesh* m, int32_t n_points, const int32_t* tet, const double* rest_xyz) {
    if (!m) return fail(VH_EINVAL, "null mesh");
    if (n_points < 0) return fail(VH_EINVAL, "n_points must be >= 0");
    if (n_points > 0 && (!tet || !rest_xyz)) return fail(VH_EINVAL, "null input arrays");
    for (int32_t i = 0; i < n_points; ++i) {
        if (tet[i] < 0 || tet[i] >= m->nt)
            return fail(VH_EINVAL, "embedded point " + std::to_string(i) + ": tet index out of range");
        for (int c = 0; c < 3; ++c)
            if (!std::isfinite(rest_xyz[3 * (size_t)i + c]))
                return fail(VH_EINVAL, "embedded point " + std::to_string(i) + ": rest position not finite");
    }
    if (m->ctx) VH_TRY(set_device(m));
    free_embedding_device(m);
    m->emb_tet.assign(tet, tet + n_points);
    m->emb_X.assign(rest_xyz, rest_xyz + 3 * (size_t)n_points);
    return VH_OK;
}

int vh_mesh_embed_device(vh_mesh* m, double* out_dev, void* stream) {
    VH_TRY(check_quiet(m));
    const int32_t n = (int32_t)m->emb_tet.size();
    if (n == 0) return VH_OK;
    if (!out_dev) return fail(VH_EINVAL, "null output");
    VH_TRY(set_device(m));
    VH_TRY(ensure_embedding(m));
    hipStream_t s = static_cast<hipStream_t>(stream);
    VH_HIP(vh::launch_embed(m->emb_rec, m->dm.x, n, out_dev, s));
    if (m->srv_id >= 0) VH_HIP(hipStreamSynchronize(s));   // ordered before the server's next frame
    return VH_OK;
}

int vh_mesh_embed(vh_mesh* m, double* out, void* stream) {
    VH_TRY(check_quiet(m));
    const int32_t n = (int32_t)m->emb_tet.size();
    if (n == 0) return VH_OK;
    if (!out) return fail(VH_EINVAL, "null output");
    VH_TRY(set_device(m));
    VH_TRY(ensure_embedding(m));
    hipStream_t s = static_cast<hipStream_t>(stream);
    VH_HIP(vh::launch_embed(m->emb_rec, m->dm.x, n, m->emb_out, s));
    VH_HIP(hipMemcpyAsync(out, m->emb_out, 3 * (size_t)n * sizeof(double), hipMemcpyDeviceToHost, s));
    VH_HIP(hipStreamSynchronize(s));
    return VH_OK;
}

}  // extern "C"
