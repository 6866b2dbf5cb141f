// Test-only host library: builds the library's host plan (partition, orderings,
// FP64 factorization, solve programs) and runs the solve programs on the CPU
// with the same semantics as the device kernels, so the plan can be checked
// against a reference solve without a GPU.  Never part of the product path.
#include <algorithm>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../paper_2405_12484_amd/csrc/plan.h"

using namespace vh;

namespace {
inline int32_t word(const float* p) {
    int32_t v;
    std::memcpy(&v, p, 4);
    return v;
}
}  // namespace

extern "C" {

void* vhp_build(const double* X, int nv, const int* tets, int nt, const double* gs, const double* gv,
                const double* mass, const unsigned char* pinned, const double* g, double dt, int iters,
                int D, int refine, int leaf_max, int* rc, char* msg, int msglen) {
    Plan* P = new Plan();
    std::string m;
    *rc = build_plan(X, nv, tets, nt, gs, gv, mass, pinned, g, dt, iters, D, refine, leaf_max, 12288, PlanOptions(), *P, m);
    std::snprintf(msg, msglen, "%s", m.c_str());
    if (*rc != 0) {
        delete P;
        return nullptr;
    }
    return P;
}

// as vhp_build, with interior chunks of at most chunk_floats 32-bit words
void* vhp_build_chunks(const double* X, int nv, const int* tets, int nt, const double* gs, const double* gv,
                       const double* mass, const unsigned char* pinned, const double* g, double dt, int iters,
                       int D, int leaf_max, int chunk_floats, int* rc, char* msg, int msglen) {
    Plan* P = new Plan();
    std::string m;
    *rc = build_plan(X, nv, tets, nt, gs, gv, mass, pinned, g, dt, iters, D, 0, leaf_max, chunk_floats, PlanOptions(),
                     *P, m);
    std::snprintf(msg, msglen, "%s", m.c_str());
    if (*rc != 0) {
        delete P;
        return nullptr;
    }
    return P;
}

void vhp_free(void* h) { delete static_cast<Plan*>(h); }

// the plan's interface factor values (host FP64 numeric factorization); their
// number, copied to out when it is not NULL
long long vhp_dvals(void* h, double* out) {
    const Plan& P = *static_cast<Plan*>(h);
    if (out) std::memcpy(out, P.dvals.data(), P.dvals.size() * sizeof(double));
    return (long long)P.dvals.size();
}

// refactor_plan with new per-element stiffness (X, tets as given to vhp_build)
void vhp_refactor(void* h, const double* X, const int* tets, const double* gs, const double* gv, int* rc, char* msg,
                  int msglen) {
    std::string m;
    *rc = refactor_plan(*static_cast<Plan*>(h), X, tets, gs, gv, m);
    std::snprintf(msg, msglen, "%s", m.c_str());
}

// sizes: n_free, n_int, n_gamma, D, n_sn, n_clevels, nnz_int, nnz_coarse, max_sub_phases,
// n_chunks, n_ctasks, n_cslots, max_sub_n
void vhp_info(void* h, long long* out) {
    const Plan& P = *static_cast<Plan*>(h);
    out[0] = P.n_free; out[1] = P.n_int; out[2] = P.n_gamma; out[3] = P.D;
    out[4] = (long long)P.sn.size(); out[5] = P.n_clevels; out[6] = P.nnz_int;
    out[7] = P.nnz_coarse; out[8] = P.max_sub_phases; out[9] = (long long)P.chunks.size();
    out[10] = (long long)P.ctasks.size(); out[11] = (long long)P.cslots.size(); out[12] = P.max_sub_n;
    out[13] = P.max_cint; out[14] = P.max_nb;
    long long mf = 0, mb = 0;   // most chunks of one subdomain's forward / backward program
    for (int d = 0; d < P.D; ++d) {
        mf = std::max<long long>(mf, P.sub_fwd_ch[d + 1] - P.sub_fwd_ch[d]);
        mb = std::max<long long>(mb, P.sub_bwd_ch[d + 1] - P.sub_bwd_ch[d]);
    }
    out[15] = mf; out[16] = mb;
}

void vhp_perm(void* h, int* perm) {
    const Plan& P = *static_cast<Plan*>(h);
    std::memcpy(perm, P.perm.data(), sizeof(int) * P.nv);
}

// Solve K_ff d = rhs; rhs, d: [nv][3] user order (pinned rows ignored / zero).
void vhp_solve(void* h, const double* rhs, double* d) {
    const Plan& P = *static_cast<Plan*>(h);
    const int nint = P.n_int, ng = P.n_gamma;
    for (int u = 0; u < P.nv * 3; ++u) d[u] = 0.0;
    for (int c = 0; c < 3; ++c) {
        std::vector<double> Rc(P.n_free), Zc(P.n_free, 0.0), Dc(P.n_free, 0.0);
        for (int i = 0; i < P.n_free; ++i) Rc[i] = rhs[3 * P.perm[i] + c];
        std::vector<double> CGF(P.n_cgf, 0.0), CGD(P.n_cgd, 0.0);
        // interior forward
        for (int s = 0; s < P.D; ++s) {
            const int base = P.sub_off[s], nloc = P.sub_off[s + 1] - base;
            std::vector<double> r(Rc.begin() + base, Rc.begin() + base + nloc), z(nloc, 0.0),
                C(P.max_cint, 0.0);
            for (int ch = P.sub_fwd_ch[s]; ch < P.sub_fwd_ch[s + 1]; ++ch) {
                const Chunk& K = P.chunks[ch];
                const float* desc = P.ivals.data() + K.v0;
                const int dw = (K.kind == PULLSUM) ? 4 : 8;
                const float* dat = desc + dw * K.ntasks;
                for (int t = 0; t < K.ntasks; ++t) {
                    const float* q = desc + dw * t;
                    if (K.kind == PULLSUM) {
                        double acc = 0.0;
                        for (int k = 0; k < word(q + 2); ++k) acc += C[word(dat + word(q + 1) + k)];
                        r[word(q)] -= acc;
                    } else {
                        const int col0 = word(q), n = word(q + 1), m = word(q + 2), mi = word(q + 3),
                                  ci0 = word(q + 4), so = word(q + 5), off = word(q + 6), row0 = word(q + 7);
                        for (int i = row0; i < std::min(row0 + 64, n + m); ++i) {
                            double acc = 0.0;
                            long co = 0;
                            const int kmax = std::min(i + 1, n);
                            for (int k = 0; k < kmax; ++k) {
                                acc += (double)dat[off + co + (i - k)] * r[col0 + k];
                                co += n + m - k;
                            }
                            if (i < n) z[col0 + i] = acc;
                            else if (i < n + mi) C[ci0 + i - n] = (double)(float)acc;
                            else CGF[word(dat + so + i - n - mi)] = (double)(float)acc;
                        }
                    }
                }
            }
            for (int i = 0; i < nloc; ++i) Zc[base + i] = z[i];
        }
        // interface forward
        std::vector<double> rg(ng, 0.0), zg(ng, 0.0), dg(ng, 0.0);
        for (const CPhase& ph : P.cfwd)
            for (int t = ph.task0; t < ph.task0 + ph.ntasks; ++t) {
                const int32_t* a = P.ctasks[t].a;
                if (ph.kind == PULLSUM) {
                    double acc = 0.0;
                    for (int k = 0; k < a[2]; ++k) acc += CGF[a[1] + k];
                    for (int k = 0; k < a[4]; ++k) acc += CGD[a[3] + k];
                    rg[a[0]] = Rc[nint + a[0]] - acc;
                } else {
                    double acc = 0.0;
                    for (int k = 0; k < a[3]; ++k) acc += P.dvals[a[2] + k] * rg[a[4] + k];
                    if (a[0] == 0) zg[a[1]] = acc;
                    else if (a[0] == 1) CGD[a[1]] = acc;
                    else dg[a[1]] = acc;
                }
            }
        // interface backward
        for (const CPhase& ph : P.cbwd)
            for (int t = ph.task0; t < ph.task0 + ph.ntasks; ++t) {
                const int32_t* a = P.ctasks[t].a;
                double acc = 0.0;
                for (int k = 0; k < a[2]; ++k) acc += P.dvals[a[1] + k] * zg[a[3] + k];
                for (int k = 0; k < a[4]; ++k) acc += P.dvals[a[1] + a[2] + k] * dg[P.cgidx[a[5] + k]];
                dg[a[0]] = acc;
            }
        for (int i = 0; i < ng; ++i) Dc[nint + i] = dg[i];
        // interior backward
        for (int s = 0; s < P.D; ++s) {
            const int base = P.sub_off[s], nloc = P.sub_off[s + 1] - base;
            const int b0 = P.bnd_off[s], nb = P.bnd_off[s + 1] - b0;
            std::vector<double> z(Zc.begin() + base, Zc.begin() + base + nloc), dl(nloc + nb, 0.0);
            for (int k = 0; k < nb; ++k) dl[nloc + k] = (double)(float)dg[P.bnd[b0 + k] - nint];
            for (int ch = P.sub_bwd_ch[s]; ch < P.sub_bwd_ch[s + 1]; ++ch) {
                const Chunk& K = P.chunks[ch];
                const float* desc = P.ivals.data() + K.v0;
                const float* dat = desc + 8 * K.ntasks;
                for (int t = 0; t < K.ntasks; ++t) {
                    const float* q = desc + 8 * t;
                    const int col0 = word(q), n = word(q + 1), m = word(q + 2), off = word(q + 3),
                              go = word(q + 4), kc0 = word(q + 5);
                    const long tri = (long)n * (n + 1) / 2;
                    for (int k = kc0; k < std::min(kc0 + 64, n); ++k) {
                        double acc = 0.0;
                        for (int i = k; i < n; ++i) acc += (double)dat[off + (long)i * (i + 1) / 2 + k] * z[col0 + i];
                        for (int pp = 0; pp < m; ++pp)
                            acc -= (double)dat[off + tri + (long)pp * n + k] * dl[word(dat + go + pp)];
                        dl[col0 + k] = acc;
                    }
                }
            }
            for (int i = 0; i < nloc; ++i) Dc[base + i] = dl[i];
        }
        for (int i = 0; i < P.n_free; ++i) d[3 * P.perm[i] + c] = Dc[i];
    }
}
}

extern "C" {
// per supernode: sub, n, m (rows below), m_interface (rows below in the interface), height, clevel
int vhp_sn_stats(void* h, int* out) {
    const Plan& P = *static_cast<Plan*>(h);
    int k = 0;
    for (const auto& s : P.sn) {
        int mg = 0;
        for (int r : s.rows) mg += (r >= P.n_int);
        out[k++] = s.sub; out[k++] = s.n; out[k++] = (int)s.rows.size(); out[k++] = mg;
        out[k++] = s.height; out[k++] = s.clevel;
    }
    return (int)P.sn.size();
}
}

extern "C" {

// as vhp_build, with the plan options (thin_separators 0/1, merge_max_cols)
void* vhp_build_opts(const double* X, int nv, const int* tets, int nt, const double* gs, const double* gv,
                     const double* mass, const unsigned char* pinned, const double* g, double dt, int iters,
                     int D, int thin, int merge, int* rc, char* msg, int msglen) {
    Plan* P = new Plan();
    std::string m;
    PlanOptions o;
    o.thin_separators = thin != 0;
    o.merge_max_cols = merge;
    *rc = build_plan(X, nv, tets, nt, gs, gv, mass, pinned, g, dt, iters, D, 0, 32, 12288, o, *P, m);
    std::snprintf(msg, msglen, "%s", m.c_str());
    if (*rc != 0) {
        delete P;
        return nullptr;
    }
    return P;
}

// interior row ranges of the subdomains (D + 1 values, internal ids)
void vhp_sub_off(void* h, int* out) {
    const Plan& P = *static_cast<Plan*>(h);
    for (size_t i = 0; i < P.sub_off.size(); ++i) out[i] = P.sub_off[i];
}

// The CMS solve as the device runs it, in FP64 from the FP32-stored modes:
// x^b from the decomposed solve's interface rows (the exact interface
// values), x^i = Phi (Lambda^{-1} Phi^T b^i) + Psi x^b per subdomain, then the
// Chebyshev-weighted Jacobi sweeps.  rhs, d: [nv][3] user order.  Returns
// build_cms's code; info[0] = rho.
int vhp_cms_solve(void* h, int modes, int sweeps, const double* rhs, double* d, double* info) {
    const Plan& P = *static_cast<Plan*>(h);
    CmsPlan C;
    std::string msg;
    int rc = build_cms(P, modes, sweeps, C, msg);
    if (rc != 0) return rc;
    info[0] = C.rho;
    const int32_t nf = P.n_free;
    std::vector<double> exact((size_t)P.nv * 3, 0.0);
    vhp_solve(h, rhs, exact.data());
    std::vector<double> b((size_t)nf * 3), x((size_t)nf * 3, 0.0);
    for (int32_t i = 0; i < nf; ++i)
        for (int c = 0; c < 3; ++c) {
            b[3 * i + c] = rhs[3 * P.perm[i] + c];
            if (i >= P.n_int) x[3 * i + c] = exact[3 * P.perm[i] + c];
        }
    for (int32_t dd = 0; dd < P.D; ++dd) {
        const int32_t r0 = P.sub_off[dd], n = P.sub_off[dd + 1] - r0;
        const int32_t b0 = P.bnd_off[dd], nb = P.bnd_off[dd + 1] - b0;
        for (int c = 0; c < 3; ++c) {
            std::vector<double> q(modes, 0.0);
            for (int k = 0; k < modes; ++k) {
                double s = 0.0;
                for (int32_t i = 0; i < n; ++i) s += (double)C.phi[C.phi_off[dd] + (size_t)k * n + i] * b[3 * (r0 + i) + c];
                q[k] = s * (double)C.ilam[(size_t)dd * modes + k];
            }
            for (int32_t i = 0; i < n; ++i) {
                double s = 0.0;
                for (int k = 0; k < modes; ++k) s += (double)C.phi[C.phi_off[dd] + (size_t)k * n + i] * q[k];
                for (int32_t j = 0; j < nb; ++j)
                    s += (double)C.psi[C.psi_off[dd] + (size_t)j * n + i] * x[3 * P.bnd[b0 + j] + c];
                x[3 * (r0 + i) + c] = s;
            }
        }
    }
    std::vector<double> prev = x, nx(x.size());
    for (int32_t k = 0; k < sweeps; ++k) {
        for (int32_t i = 0; i < nf; ++i)
            for (int c = 0; c < 3; ++c) {
                double s = 0.0;
                for (int32_t t = P.K_ptr[i]; t < P.K_ptr[i + 1]; ++t) s += P.K_val[t] * x[3 * P.K_col[t] + c];
                const double xh = x[3 * i + c] + C.inv_diag[i] * (b[3 * i + c] - s);
                nx[3 * i + c] = C.omega[k] * (xh - prev[3 * i + c]) + prev[3 * i + c];
            }
        prev.swap(x);
        x.swap(nx);
    }
    std::fill(d, d + (size_t)P.nv * 3, 0.0);
    for (int32_t i = 0; i < nf; ++i)
        for (int c = 0; c < 3; ++c) d[3 * P.perm[i] + c] = x[3 * i + c];
    return 0;
}

}  // extern "C"
