// Test-only host library: builds the library's host plan (partition, orderings,
// FP64 factorization, solve programs) and runs the solve programs on the CPU
// with the same semantics as the device kernels, so the plan can be checked
// against a reference solve without a GPU.  Never part of the product path.
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../paper_2405_12484_amd/csrc/plan.h"

using namespace vh;

namespace {

template <class T>
double seg_dot(const Plan& P, const Seg& g, const T* x) {
    double acc = 0.0;
    if (g.kind == 1)
        for (int k = 0; k < g.len; ++k) acc += (double)P.fvals[g.voff + k] * (double)x[g.xoff + k];
    else
        for (int k = 0; k < g.len; ++k) acc += P.dvals[g.voff + k] * (double)x[g.xoff + k];
    return acc;
}

}  // namespace

extern "C" {

void* vhp_build(const double* X, int nv, const int* tets, int nt, const double* gs, const double* gv,
                const double* mass, const unsigned char* pinned, const double* g, double dt, int iters,
                int D, int refine, int leaf_max, int* rc, char* msg, int msglen) {
    Plan* P = new Plan();
    std::string m;
    *rc = build_plan(X, nv, tets, nt, gs, gv, mass, pinned, g, dt, iters, D, refine, leaf_max, 4096, *P, m);
    std::snprintf(msg, msglen, "%s", m.c_str());
    if (*rc != 0) {
        delete P;
        return nullptr;
    }
    return P;
}

void vhp_free(void* h) { delete static_cast<Plan*>(h); }

// sizes: n_free, n_int, n_gamma, D, n_sn, n_clevels, nnz_int, nnz_coarse, max_sub_phases,
// n_phases, n_tasks, n_segs, max_sub_n
void vhp_info(void* h, long long* out) {
    const Plan& P = *static_cast<Plan*>(h);
    out[0] = P.n_free; out[1] = P.n_int; out[2] = P.n_gamma; out[3] = P.D;
    out[4] = (long long)P.sn.size(); out[5] = P.n_clevels; out[6] = P.nnz_int;
    out[7] = P.nnz_coarse; out[8] = P.max_sub_phases; out[9] = (long long)P.phases.size();
    out[10] = (long long)P.tasks.size(); out[11] = (long long)P.segs.size(); out[12] = P.max_sub_n;
}

void vhp_perm(void* h, int* perm) {
    const Plan& P = *static_cast<Plan*>(h);
    std::memcpy(perm, P.perm.data(), sizeof(int) * P.nv);
}

// Solve K_ff d = rhs; rhs, d: [nv][3] user order (pinned rows ignored / zero).
void vhp_solve(void* h, const double* rhs, double* d) {
    const Plan& P = *static_cast<Plan*>(h);
    const int nint = P.n_int, ng = P.n_gamma;
    std::vector<double> R((size_t)P.n_free * 3), Z((size_t)P.n_free * 3), Dv((size_t)P.n_free * 3);
    for (int i = 0; i < P.n_free; ++i)
        for (int c = 0; c < 3; ++c) R[3 * i + c] = rhs[3 * P.perm[i] + c];
    for (int c = 0; c < 3; ++c) {
        std::vector<double> Rc(P.n_free), Zc(P.n_free, 0.0), Dc(P.n_free, 0.0);
        for (int i = 0; i < P.n_free; ++i) Rc[i] = R[3 * i + c];
        // interior forward (chunk programs, values from ivals)
        for (int s = 0; s < P.D; ++s) {
            const int base = P.sub_off[s], nloc = P.sub_off[s + 1] - base;
            std::vector<double> r(Rc.begin() + base, Rc.begin() + base + nloc), z(nloc, 0.0);
            for (int ch = P.sub_fwd_ch[s]; ch < P.sub_fwd_ch[s + 1]; ++ch) {
                const Chunk& C = P.chunks[ch];
                const float* cur = P.ivals.data() + C.v0;
                for (int t = C.task0; t < C.task1; ++t) {
                    const Task& T = P.tasks[t];
                    double acc = 0.0;
                    for (int g = T.seg0; g < T.seg1; ++g) {
                        const Seg& S = P.segs[g];
                        const std::vector<double>& xv = (C.kind == FWD_PULL) ? z : r;
                        for (int k = 0; k < S.len; ++k) acc += (double)cur[S.voff + k] * xv[S.xoff + k];
                    }
                    if (C.kind == FWD_PULL) r[T.out] -= acc;
                    else z[T.out] = acc;
                }
            }
            for (int i = 0; i < nloc; ++i) Zc[base + i] = z[i];
        }
        // interface forward
        std::vector<double> R64(Rc.begin() + nint, Rc.end()), Z64(ng, 0.0), D64(ng, 0.0);
        for (int ph : P.coarse_fwd_ph) {
            const Phase& Ph = P.phases[ph];
            std::vector<double> outv(Ph.task1 - Ph.task0);
            for (int t = Ph.task0; t < Ph.task1; ++t) {
                const Task& T = P.tasks[t];
                double acc = 0.0;
                for (int g = T.seg0; g < T.seg1; ++g) {
                    const Seg& S = P.segs[g];
                    if (Ph.kind == FWD_PULL) acc += seg_dot(P, S, S.kind == 1 ? Zc.data() : Z64.data());
                    else acc += seg_dot(P, S, R64.data());
                }
                outv[t - Ph.task0] = (Ph.kind == FWD_PULL) ? R64[T.out] - acc : acc;
            }
            for (int t = Ph.task0; t < Ph.task1; ++t) {
                const Task& T = P.tasks[t];
                if (Ph.kind == FWD_PULL) R64[T.out] = outv[t - Ph.task0];
                else Z64[T.out] = outv[t - Ph.task0];
            }
        }
        // interface backward
        for (int ph : P.coarse_bwd_ph) {
            const Phase& Ph = P.phases[ph];
            std::vector<double> outv(Ph.task1 - Ph.task0);
            for (int t = Ph.task0; t < Ph.task1; ++t) {
                const Task& T = P.tasks[t];
                double acc = 0.0;
                for (int g = T.seg0; g < T.seg1; ++g) {
                    const Seg& S = P.segs[g];
                    if (Ph.kind == BWD_PULL) {
                        for (int k = 0; k < S.len; ++k)
                            acc += P.dvals[S.voff + k] * D64[P.gidx[S.xoff + k] - nint];
                    } else {
                        acc += seg_dot(P, S, R64.data());
                    }
                }
                outv[t - Ph.task0] = (Ph.kind == BWD_PULL) ? Z64[T.out] - acc : acc;
            }
            for (int t = Ph.task0; t < Ph.task1; ++t) {
                const Task& T = P.tasks[t];
                if (Ph.kind == BWD_PULL) R64[T.out] = outv[t - Ph.task0];
                else D64[T.out] = outv[t - Ph.task0];
            }
        }
        for (int i = 0; i < ng; ++i) Dc[nint + i] = D64[i];
        // interior backward (chunk programs, gathers through the staged boundary rows)
        for (int s = 0; s < P.D; ++s) {
            const int base = P.sub_off[s], nloc = P.sub_off[s + 1] - base;
            const int b0 = P.bnd_off[s], nb = P.bnd_off[s + 1] - b0;
            std::vector<double> zq(Zc.begin() + base, Zc.begin() + base + nloc), dl(nloc + nb, 0.0);
            for (int k = 0; k < nb; ++k) dl[nloc + k] = (double)(float)D64[P.bnd[b0 + k] - nint];
            for (int ch = P.sub_bwd_ch[s]; ch < P.sub_bwd_ch[s + 1]; ++ch) {
                const Chunk& C = P.chunks[ch];
                const float* cur = P.ivals.data() + C.v0;
                for (int t = C.task0; t < C.task1; ++t) {
                    const Task& T = P.tasks[t];
                    double acc = 0.0;
                    for (int g = T.seg0; g < T.seg1; ++g) {
                        const Seg& S = P.segs[g];
                        for (int k = 0; k < S.len; ++k) {
                            if (C.kind == BWD_PULL) {
                                int li;
                                std::memcpy(&li, cur + S.xoff + k, 4);
                                acc += (double)cur[S.voff + k] * dl[li];
                            } else {
                                acc += (double)cur[S.voff + k] * zq[S.xoff + k];
                            }
                        }
                    }
                    if (C.kind == BWD_PULL) zq[T.out] -= acc;
                    else dl[T.out] = acc;
                }
            }
            for (int i = 0; i < nloc; ++i) Dc[base + i] = dl[i];
        }
        for (int i = 0; i < P.n_free; ++i) Dv[3 * i + c] = Dc[i];
    }
    for (int u = 0; u < P.nv * 3; ++u) d[u] = 0.0;
    for (int i = 0; i < P.n_free; ++i)
        for (int c = 0; c < 3; ++c) d[3 * P.perm[i] + c] = Dv[3 * i + c];
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
