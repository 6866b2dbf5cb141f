// Host prefactor of the decomposed PD global step (FP64).
//
// The global matrix of the PD global step (Sec. 7.1) is constant, so it is
// factored once per material.  Because row c of F_e depends only on
// coordinate c of the corners, the 3n x 3n matrix K is L (x) I_3 with the
// scalar L = M/dt^2 + sum_e V_e (gs_e + gv_e) G_e, (G_e)_ab = gradN_a . gradN_b;
// every solve here is a scalar solve with three right-hand-side columns.
//
// Domain decomposition (Sec. 7.2): the elements are split into subdomains, the
// free vertices touched by one subdomain are its internal DOFs, the rest are
// boundary (interface) DOFs shared by neighbours -- the paper's duplicated
// boundary DOFs made unique as in Eq. (global_subspace).  With the interior
// unknowns ordered first, block elimination gives the interior factors and the
// interface Schur complement S = K^bb - sum_d K_d^bi (K_d^ii)^{-1} K_d^ib, which
// is what the reduced system of the paper's boundary modes
// Psi_d = -(K_d^ii)^{-1} K_d^ib (Eq. cms_boundary) becomes when the interior
// eigenmodes are replaced by exact interior solves.  The interface is ordered
// by the bisection tree (each interface vertex goes to the lowest tree node
// whose subtree holds every subdomain touching it) and each interior by nested
// dissection, so the whole factor is one supernodal tree: per supernode a dense
// diagonal block (stored inverted, so the device solves are dot products
// without a sequential chain) and a dense block of rows below it.
#include "plan.h"

#include <omp.h>

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <chrono>
#include <cmath>
#include <cstring>
#include <numeric>

namespace vh {

namespace {

constexpr int OK = 0, EINVAL_ = -1, ENOMEM_ = -2, ENOTSPD_ = -3;
// Interior supernodes have at most this many columns, so that one supernode's
// solve block fits an LDS chunk and a wave's lanes cover its columns.
constexpr int32_t kMaxInteriorCols = 32;
// tets per local-step workgroup (one thread per tet)
constexpr int32_t kLocalBlock = 256;

inline void tet_dm(const double* X, const int32_t* t, double Dm[9]) {
    // Dm[r][k] = X[t[k+1]][r] - X[t[0]][r]
    for (int r = 0; r < 3; ++r)
        for (int k = 0; k < 3; ++k) Dm[r * 3 + k] = X[t[k + 1] * 3 + r] - X[t[0] * 3 + r];
}

inline double det3(const double* A) {
    return A[0] * (A[4] * A[8] - A[5] * A[7]) - A[1] * (A[3] * A[8] - A[5] * A[6]) +
           A[2] * (A[3] * A[7] - A[4] * A[6]);
}

inline void inv3(const double* A, double det, double* B) {
    double id = 1.0 / det;
    B[0] = (A[4] * A[8] - A[5] * A[7]) * id;
    B[1] = (A[2] * A[7] - A[1] * A[8]) * id;
    B[2] = (A[1] * A[5] - A[2] * A[4]) * id;
    B[3] = (A[5] * A[6] - A[3] * A[8]) * id;
    B[4] = (A[0] * A[8] - A[2] * A[6]) * id;
    B[5] = (A[2] * A[3] - A[0] * A[5]) * id;
    B[6] = (A[3] * A[7] - A[4] * A[6]) * id;
    B[7] = (A[1] * A[6] - A[0] * A[7]) * id;
    B[8] = (A[0] * A[4] - A[1] * A[3]) * id;
}

// ---------------------------------------------------------------------------
// Element partition: recursive breadth-first bisection of the face graph.
// ---------------------------------------------------------------------------
void face_adjacency(int32_t nt, const int32_t* tets, std::vector<int32_t>& ptr,
                    std::vector<int32_t>& adj) {
    struct Face {
        int32_t a, b, c, e;
    };
    std::vector<Face> faces((size_t)nt * 4);
    for (int32_t e = 0; e < nt; ++e) {
        int32_t v[4] = {tets[4 * e], tets[4 * e + 1], tets[4 * e + 2], tets[4 * e + 3]};
        std::sort(v, v + 4);
        faces[4 * (size_t)e + 0] = {v[0], v[1], v[2], e};
        faces[4 * (size_t)e + 1] = {v[0], v[1], v[3], e};
        faces[4 * (size_t)e + 2] = {v[0], v[2], v[3], e};
        faces[4 * (size_t)e + 3] = {v[1], v[2], v[3], e};
    }
    std::sort(faces.begin(), faces.end(), [](const Face& x, const Face& y) {
        if (x.a != y.a) return x.a < y.a;
        if (x.b != y.b) return x.b < y.b;
        if (x.c != y.c) return x.c < y.c;
        return x.e < y.e;
    });
    std::vector<std::pair<int32_t, int32_t>> pairs;
    for (size_t i = 0; i + 1 < faces.size(); ++i) {
        const Face& f = faces[i];
        const Face& g = faces[i + 1];
        if (f.a == g.a && f.b == g.b && f.c == g.c) {
            pairs.push_back({f.e, g.e});
            pairs.push_back({g.e, f.e});
        }
    }
    std::sort(pairs.begin(), pairs.end());
    ptr.assign(nt + 1, 0);
    adj.resize(pairs.size());
    for (size_t i = 0; i < pairs.size(); ++i) {
        ptr[pairs[i].first + 1]++;
        adj[i] = pairs[i].second;
    }
    for (int32_t i = 0; i < nt; ++i) ptr[i + 1] += ptr[i];
}

// BFS over elements with part[e] == p, from `start`, continuing from the
// lowest unvisited member when a component ends.  members: ascending.
void bfs_part(int32_t start, int32_t p, const std::vector<int32_t>& members,
              const std::vector<int32_t>& part, const std::vector<int32_t>& ptr,
              const std::vector<int32_t>& adj, std::vector<int32_t>& stamp, int32_t tok,
              std::vector<int32_t>& order) {
    order.clear();
    order.reserve(members.size());
    size_t head = 0, mi = 0;
    stamp[start] = tok;
    order.push_back(start);
    while (order.size() < members.size()) {
        while (head < order.size()) {
            int32_t u = order[head++];
            for (int32_t k = ptr[u]; k < ptr[u + 1]; ++k) {
                int32_t w = adj[k];
                if (part[w] == p && stamp[w] != tok) {
                    stamp[w] = tok;
                    order.push_back(w);
                }
            }
        }
        while (order.size() < members.size() && mi < members.size()) {
            int32_t c = members[mi++];
            if (stamp[c] != tok) {
                stamp[c] = tok;
                order.push_back(c);
                break;
            }
        }
    }
}

std::vector<int32_t> bisect_elements(int32_t nt, const int32_t* tets, int32_t D) {
    std::vector<int32_t> ptr, adj;
    face_adjacency(nt, tets, ptr, adj);
    std::vector<int32_t> part(nt, 0), next(nt, 0), stamp(nt, -1), order, order2;
    int32_t tok = 0;
    for (int32_t nparts = 1; nparts < D; nparts *= 2) {
        std::vector<std::vector<int32_t>> members(nparts);
        for (int32_t e = 0; e < nt; ++e) members[part[e]].push_back(e);
        for (int32_t p = 0; p < nparts; ++p) {
            const auto& M = members[p];
            if (M.empty()) continue;
            bfs_part(M[0], p, M, part, ptr, adj, stamp, ++tok, order);
            bfs_part(order.back(), p, M, part, ptr, adj, stamp, ++tok, order2);
            size_t h = order2.size() / 2;
            for (size_t i = 0; i < order2.size(); ++i) next[order2[i]] = 2 * p + (i < h ? 0 : 1);
        }
        part.swap(next);
    }
    return part;
}

// ---------------------------------------------------------------------------
// Nested dissection of one subdomain's interior vertices.
// ---------------------------------------------------------------------------
struct NDNode {
    std::vector<int32_t> verts;
    int32_t left = -1, right = -1;
};

struct NDScratch {
    std::vector<int32_t> mark, level;
    int32_t tok = 0;
};

// BFS inside the set marked with `tok`; returns the visit order of the component.
void bfs_set(int32_t s, int32_t tok, const std::vector<int32_t>& vptr,
             const std::vector<int32_t>& vadj, NDScratch& sc, int32_t vtok,
             std::vector<int32_t>& order) {
    // mark[v] == tok: in the set and unvisited; set to vtok when visited
    order.clear();
    sc.mark[s] = vtok;
    sc.level[s] = 0;
    order.push_back(s);
    size_t head = 0;
    while (head < order.size()) {
        int32_t u = order[head++];
        for (int32_t k = vptr[u]; k < vptr[u + 1]; ++k) {
            int32_t w = vadj[k];
            if (sc.mark[w] == tok) {
                sc.mark[w] = vtok;
                sc.level[w] = sc.level[u] + 1;
                order.push_back(w);
            }
        }
    }
    for (int32_t v : order) sc.mark[v] = tok;   // restore set membership
}

int32_t nd_build(std::vector<int32_t> S, int32_t leaf_max, const std::vector<int32_t>& vptr,
                 const std::vector<int32_t>& vadj, NDScratch& sc, std::vector<NDNode>& T) {
    int32_t id = (int32_t)T.size();
    T.emplace_back();
    if ((int32_t)S.size() <= leaf_max) {
        std::sort(S.begin(), S.end());
        T[id].verts = std::move(S);
        return id;
    }
    int32_t tok = ++sc.tok;
    int32_t vtok = ++sc.tok;
    for (int32_t v : S) sc.mark[v] = tok;
    int32_t smin = *std::min_element(S.begin(), S.end());
    std::vector<int32_t> order;
    bfs_set(smin, tok, vptr, vadj, sc, vtok, order);
    std::vector<int32_t> A, B, sep;
    if (order.size() < S.size()) {
        // disconnected: first component versus the rest, no separator needed
        int32_t ctok = ++sc.tok;
        for (int32_t v : order) sc.mark[v] = ctok;
        A = order;
        for (int32_t v : S)
            if (sc.mark[v] != ctok) B.push_back(v);
    } else {
        int32_t far = order.back();
        vtok = ++sc.tok;
        bfs_set(far, tok, vptr, vadj, sc, vtok, order);
        int32_t maxlev = 0;
        for (int32_t v : order) maxlev = std::max(maxlev, sc.level[v]);
        std::vector<int32_t> cnt(maxlev + 2, 0);
        for (int32_t v : order) cnt[sc.level[v]]++;
        int32_t cum = 0, cut = maxlev;
        for (int32_t l = 0; l <= maxlev; ++l) {
            cum += cnt[l];
            if (2 * cum >= (int32_t)S.size()) {
                cut = l;
                break;
            }
        }
        if (cut == 0) cut = std::min(1, maxlev);
        for (int32_t v : order) {
            int32_t l = sc.level[v];
            if (l < cut) A.push_back(v);
            else if (l == cut) sep.push_back(v);
            else B.push_back(v);
        }
    }
    for (int32_t v : S) sc.mark[v] = 0;
    std::sort(sep.begin(), sep.end());
    T[id].verts = std::move(sep);
    int32_t l = A.empty() ? -1 : nd_build(std::move(A), leaf_max, vptr, vadj, sc, T);
    int32_t r = B.empty() ? -1 : nd_build(std::move(B), leaf_max, vptr, vadj, sc, T);
    T[id].left = l;
    T[id].right = r;
    return id;
}

// ---------------------------------------------------------------------------
// Dense kernels for the multifrontal factorization (column-major fronts).
// ---------------------------------------------------------------------------
// Factor the first n columns of the f x f symmetric front F (lower part,
// column-major): F11 = L11 L11^T, L21 = F21 L11^{-T}, F22 -= L21 L21^T.
int partial_cholesky(double* F, int32_t f, int32_t n, bool par) {
    const int32_t NB = 32;
    for (int32_t k0 = 0; k0 < n; k0 += NB) {
        int32_t kb = std::min(NB, n - k0);
        for (int32_t k = k0; k < k0 + kb; ++k) {
            double* ck = F + (size_t)k * f;
            double piv = ck[k];
            if (!(piv > 0.0) || !std::isfinite(piv)) return ENOTSPD_;
            double l = std::sqrt(piv);
            ck[k] = l;
            double il = 1.0 / l;
            for (int32_t i = k + 1; i < f; ++i) ck[i] *= il;
            for (int32_t j = k + 1; j < k0 + kb; ++j) {
                double a = ck[j];
                double* cj = F + (size_t)j * f;
                for (int32_t i = j; i < f; ++i) cj[i] -= ck[i] * a;
            }
        }
        int32_t j0 = k0 + kb;
        auto update = [&](int32_t j) {
            double* cj = F + (size_t)j * f;
            for (int32_t k = k0; k < k0 + kb; ++k) {
                const double* ck = F + (size_t)k * f;
                double a = ck[j];
                if (a == 0.0) continue;
                for (int32_t i = j; i < f; ++i) cj[i] -= ck[i] * a;
            }
        };
        if (par && (int64_t)(f - j0) * (f - j0) > 200000) {
#pragma omp parallel for schedule(dynamic, 8)
            for (int32_t j = j0; j < f; ++j) update(j);
        } else {
            for (int32_t j = j0; j < f; ++j) update(j);
        }
    }
    return OK;
}

// Inverse of the n x n lower-triangular L (column-major with leading dim f)
// into Ti (row-major n x n, lower part).
void lower_inverse(const double* L, int32_t f, int32_t n, std::vector<double>& Ti, bool par) {
    Ti.assign((size_t)n * n, 0.0);
    auto col = [&](int32_t j) {
        // solve L x = e_j (x[i] = 0 for i < j) column by column of L, each
        // column read contiguously
        std::vector<double> x(n, 0.0);
        x[j] = 1.0;
        for (int32_t k = j; k < n; ++k) {
            const double* lk = L + (size_t)k * f;
            const double xk = x[k] / lk[k];
            x[k] = xk;
            if (xk == 0.0) continue;
            for (int32_t i = k + 1; i < n; ++i) x[i] -= lk[i] * xk;
        }
        for (int32_t i = j; i < n; ++i) Ti[(size_t)i * n + j] = x[i];
    };
    if (par && n > 128) {
#pragma omp parallel for schedule(dynamic, 4)
        for (int32_t j = 0; j < n; ++j) col(j);
    } else {
        for (int32_t j = 0; j < n; ++j) col(j);
    }
}

// K on the free unknowns in internal order (CSR, columns ascending):
// sum_e V_e (gs_e + gv_e) (G_e)_ab plus M/dt^2 on the diagonal (Sec. 7.1).
// Vol, Gd: per internal element its volume and Dm^{-1} (row-major).  The
// pattern, and the entry each (element, corner pair) adds to, are found once;
// the values are then summed in element order (a refactorization repeats
// only that, in the same order).
void assemble_matrix(Plan& P, const std::vector<double>& Vol, const std::vector<double>& Gd, const double* gamma_s,
                     const double* gamma_v, double dt) {
    const int32_t nf = P.n_free, nt = P.nt;
    if (P.K_pair.empty()) {
        std::vector<std::vector<int32_t>> rows(nf);
        for (int32_t e = 0; e < nt; ++e)
            for (int a = 0; a < 4; ++a) {
                const int32_t ia = P.tet_soa[(size_t)a * nt + e];
                if (ia >= nf) continue;
                for (int b = 0; b < 4; ++b) {
                    const int32_t ib = P.tet_soa[(size_t)b * nt + e];
                    if (ib < nf) rows[ia].push_back(ib);
                }
            }
        P.K_ptr.assign(nf + 1, 0);
        for (int32_t i = 0; i < nf; ++i) {
            auto& r = rows[i];
            r.push_back(i);
            std::sort(r.begin(), r.end());
            r.erase(std::unique(r.begin(), r.end()), r.end());
            P.K_ptr[i + 1] = P.K_ptr[i] + (int32_t)r.size();
        }
        P.K_col.resize(P.K_ptr[nf]);
        for (int32_t i = 0; i < nf; ++i) std::copy(rows[i].begin(), rows[i].end(), P.K_col.begin() + P.K_ptr[i]);
        auto at = [&](int32_t i, int32_t j) {
            const auto b0 = P.K_col.begin() + P.K_ptr[i], b1 = P.K_col.begin() + P.K_ptr[i + 1];
            return (int32_t)(std::lower_bound(b0, b1, j) - P.K_col.begin());
        };
        P.K_diag.resize(nf);
        for (int32_t i = 0; i < nf; ++i) P.K_diag[i] = at(i, i);
        P.K_pair.assign((size_t)nt * 16, -1);
        for (int32_t e = 0; e < nt; ++e)
            for (int a = 0; a < 4; ++a) {
                const int32_t ia = P.tet_soa[(size_t)a * nt + e];
                if (ia >= nf) continue;
                for (int b = 0; b < 4; ++b) {
                    const int32_t ib = P.tet_soa[(size_t)b * nt + e];
                    if (ib < nf) P.K_pair[(size_t)e * 16 + a * 4 + b] = at(ia, ib);
                }
            }
    }
    P.K_val.assign(P.K_col.size(), 0.0);
    for (int32_t i = 0; i < nf; ++i) P.K_val[P.K_diag[i]] = P.mass_int[i] / (dt * dt);
    for (int32_t e = 0; e < nt; ++e) {
        double gr[4][3];
        const double* G = &Gd[(size_t)e * 9];
        for (int k = 0; k < 3; ++k) {
            gr[0][k] = -(G[0 * 3 + k] + G[1 * 3 + k] + G[2 * 3 + k]);
            for (int c = 1; c < 4; ++c) gr[c][k] = G[(c - 1) * 3 + k];
        }
        const int32_t u = P.elem_perm[e];
        const double w = Vol[e] * (gamma_s[u] + gamma_v[u]);
        const int32_t* kp = &P.K_pair[(size_t)e * 16];
        for (int a = 0; a < 4; ++a)
            for (int b = 0; b < 4; ++b) {
                const int32_t k = kp[a * 4 + b];
                if (k < 0) continue;
                P.K_val[k] += w * (gr[a][0] * gr[b][0] + gr[a][1] * gr[b][1] + gr[a][2] * gr[b][2]);
            }
    }
}

// Numeric multifrontal FP64 factorization of P's matrix over its supernodes
// (rows below and value offsets already set): the value blocks of interior
// supernodes go to ivd (P.n_ivd values), those of interface supernodes to
// P.dvals.  Interior subdomains in parallel; interface supernodes in order,
// each with parallel dense kernels.  OK, or ENOTSPD_ with msg set.
int factor_numeric(Plan& P, std::vector<double>& ivd, std::string& msg) {
    std::vector<Supernode>& SN = P.sn;
    const int32_t nsn = (int32_t)SN.size(), nf = P.n_free, D = P.D;
    std::vector<std::vector<double>> upd(nsn);
    int err = OK;
    auto numeric = [&](int32_t t, std::vector<int32_t>& pos, bool par) -> int {
        Supernode& s = SN[t];
        const int32_t n = s.n, m = (int32_t)s.rows.size(), f = n + m;
        std::vector<double> F((size_t)f * f, 0.0);
        for (int32_t a = 0; a < n; ++a) pos[s.col0 + a] = a;
        for (int32_t b = 0; b < m; ++b) pos[s.rows[b]] = n + b;
        for (int32_t a = 0; a < n; ++a) {
            int32_t j = s.col0 + a;
            for (int32_t k = P.K_ptr[j]; k < P.K_ptr[j + 1]; ++k) {
                int32_t i = P.K_col[k];
                if (i < j) continue;
                F[(size_t)a * f + pos[i]] += P.K_val[k];
            }
        }
        for (int32_t c : s.children) {
            const Supernode& cs = SN[c];
            const int32_t mc = (int32_t)cs.rows.size();
            const std::vector<double>& U = upd[c];
            for (int32_t b2 = 0; b2 < mc; ++b2) {
                int32_t pb = pos[cs.rows[b2]];
                for (int32_t a2 = b2; a2 < mc; ++a2)
                    F[(size_t)pb * f + pos[cs.rows[a2]]] += U[(size_t)b2 * mc + a2];
            }
            std::vector<double>().swap(upd[c]);
        }
        int rc = partial_cholesky(F.data(), f, n, par);
        if (rc != OK) return rc;
        std::vector<double> Ti;
        lower_inverse(F.data(), f, n, Ti, par);
        // W_B[p][a] = sum_{b >= a} B[p][b] Ti[b][a], B[p][b] = F(n + p, b)
        std::vector<double> WB((size_t)m * n, 0.0);
        auto wrow = [&](int32_t p) {
            for (int32_t b = 0; b < n; ++b) {
                const double bv = F[(size_t)b * f + n + p];
                if (bv == 0.0) continue;
                const double* tr = &Ti[(size_t)b * n];
                double* wr = &WB[(size_t)p * n];
                for (int32_t a = 0; a <= b; ++a) wr[a] += bv * tr[a];
            }
        };
        if (par && (int64_t)m * n * n > 4000000) {
#pragma omp parallel for schedule(dynamic, 4)
            for (int32_t p = 0; p < m; ++p) wrow(p);
        } else {
            for (int32_t p = 0; p < m; ++p) wrow(p);
        }
        double* vals = (s.sub >= 0) ? ivd.data() : P.dvals.data();
        const int64_t tri = (int64_t)n * (n + 1) / 2;
        if (s.sub < 0 && m == 0) {
            // an interface root (no rows below): its forward and backward
            // solves compose to d = Ti^T Ti r', so the full symmetric
            // A = Ti^T Ti (n^2 <= 2 tri values, both layouts' space) is stored
            // row-major and applied in one pass.  A[i][j] = sum_{k >= max(i, j)}
            // Ti[k][i] Ti[k][j], dot products of Ti's columns.
            std::vector<double> TC((size_t)n * n, 0.0);   // TC[i][k] = Ti[k][i]
            for (int32_t k = 0; k < n; ++k)
                for (int32_t i = 0; i <= k; ++i) TC[(size_t)i * n + k] = Ti[(size_t)k * n + i];
            double* A = vals + s.wf_off;
#pragma omp parallel for schedule(dynamic, 8) if (par)
            for (int32_t i = 0; i < n; ++i) {
                const double* ci = &TC[(size_t)i * n];
                for (int32_t j = i; j < n; ++j) {
                    const double* cj = &TC[(size_t)j * n];
                    double acc = 0.0;
                    for (int32_t k = j; k < n; ++k) acc += ci[k] * cj[k];
                    A[(int64_t)i * n + j] = acc;
                    A[(int64_t)j * n + i] = acc;
                }
            }
            upd[t].clear();
            return OK;
        }
        for (int32_t a = 0; a < n; ++a)
            for (int32_t b = 0; b <= a; ++b) vals[s.wf_off + (int64_t)a * (a + 1) / 2 + b] = Ti[(size_t)a * n + b];
        for (int32_t p = 0; p < m; ++p)
            for (int32_t a = 0; a < n; ++a) vals[s.wf_off + tri + (int64_t)p * n + a] = WB[(size_t)p * n + a];
        for (int32_t k = 0; k < n; ++k) {
            int64_t off = s.wb_off + (int64_t)k * (n + m) - (int64_t)k * (k - 1) / 2;
            for (int32_t i = k; i < n; ++i) vals[off + (i - k)] = Ti[(size_t)i * n + k];
            off += n - k;
            // interface blocks hold -W_B (backward dot products); interior blocks +W_B
            const double sg = (s.sub >= 0) ? 1.0 : -1.0;
            for (int32_t p = 0; p < m; ++p) vals[off + p] = sg * WB[(size_t)p * n + k];
        }
        std::vector<double> U((size_t)m * m);
        for (int32_t b = 0; b < m; ++b)
            for (int32_t a = b; a < m; ++a) U[(size_t)b * m + a] = F[(size_t)(n + b) * f + n + a];
        upd[t] = std::move(U);
        return OK;
    };
#pragma omp parallel
    {
        std::vector<int32_t> pos(nf, 0);
#pragma omp for schedule(dynamic, 1)
        for (int32_t d = 0; d < D; ++d) {
            for (int32_t t = 0; t < nsn; ++t) {
                if (SN[t].sub != d) continue;
                int rc = numeric(t, pos, false);
                if (rc != OK) {
#pragma omp critical
                    err = rc;
                    break;
                }
            }
        }
    }
    if (err != OK) {
        msg = "non-positive pivot in an interior factor";
        return err;
    }
    if (P.iface_on_device) {
        // the interior contributions to interface fronts wait for the device
        P.iface_child_upd.assign(nsn, {});
        for (int32_t t = 0; t < nsn; ++t)
            if (SN[t].sub >= 0 && SN[t].parent >= 0 && SN[SN[t].parent].sub < 0)
                P.iface_child_upd[t] = std::move(upd[t]);
        P.dvals_ready = false;
        return OK;
    }
    {
        std::vector<int32_t> pos(nf, 0);
        for (int32_t t = 0; t < nsn; ++t) {
            if (SN[t].sub >= 0) continue;
            int rc = numeric(t, pos, true);
            if (rc != OK) {
                msg = "non-positive pivot in the interface factor";
                return rc;
            }
        }
    }
    P.dvals_ready = true;
    return OK;
}

}  // namespace

int check_mesh(const double* X, int32_t nv, const int32_t* tets, int32_t nt, std::string& msg) {
    if (nv <= 0 || nt <= 0 || !X || !tets) {
        msg = "empty mesh";
        return EINVAL_;
    }
    for (int32_t e = 0; e < nt; ++e) {
        for (int c = 0; c < 4; ++c) {
            int32_t v = tets[4 * e + c];
            if (v < 0 || v >= nv) {
                msg = "tet " + std::to_string(e) + " has a vertex id out of range";
                return EINVAL_;
            }
        }
        double Dm[9];
        tet_dm(X, tets + 4 * e, Dm);
        double vol = det3(Dm) / 6.0;
        if (!(vol > 0.0)) {
            msg = "tet " + std::to_string(e) + " has non-positive rest volume";
            return EINVAL_;
        }
    }
    return OK;
}

int build_plan(const double* X, int32_t nv, const int32_t* tets, int32_t nt,
               const double* gamma_s, const double* gamma_v, const double* mass,
               const uint8_t* pinned, const double* gravity, double dt, int32_t pd_iters,
               int32_t D, int32_t refine_steps, int32_t leaf_max, int32_t chunk_floats,
               const PlanOptions& opt, Plan& P, std::string& msg) {
    auto t_start = std::chrono::steady_clock::now();
    if (D < 1 || (D & (D - 1))) {
        msg = "n_subdomains must be a power of two >= 1";
        return EINVAL_;
    }
    if (D > nt) {
        msg = "more subdomains than elements";
        return EINVAL_;
    }
    P = Plan();
    P.nv = nv;
    P.nt = nt;
    P.D = D;
    P.dt = dt;
    P.pd_iters = pd_iters;
    P.refine_steps = refine_steps;
    for (int c = 0; c < 3; ++c) P.gravity[c] = gravity[c];
    P.pinned_user.assign(pinned, pinned + nv);

    // ---- partition and vertex classes --------------------------------------
    std::vector<int32_t> part = bisect_elements(nt, tets, D);
    int32_t kbits = 0;
    while ((1 << kbits) < D) ++kbits;
    std::vector<int32_t> first(nv, -1), xr(nv, 0);
    for (int32_t e = 0; e < nt; ++e)
        for (int c = 0; c < 4; ++c) {
            int32_t v = tets[4 * e + c];
            if (first[v] < 0) first[v] = part[e];
            else xr[v] |= (part[e] ^ first[v]);
        }
    // heap node of each free vertex: D + p for interior of p, the LCA node otherwise
    std::vector<int32_t> node(nv, -1);
    for (int32_t v = 0; v < nv; ++v) {
        if (pinned[v] || first[v] < 0) continue;
        if (xr[v] == 0) {
            node[v] = D + first[v];
        } else {
            int32_t bl = 32 - __builtin_clz((uint32_t)xr[v]);
            int32_t lvl = kbits - bl;             // depth of the LCA
            node[v] = (1 << lvl) + (first[v] >> bl);
        }
    }
    for (int32_t v = 0; v < nv; ++v)
        if (!pinned[v] && first[v] < 0) {
            msg = "free vertex " + std::to_string(v) + " belongs to no element";
            return EINVAL_;
        }
    // ---- vertex adjacency ------------------------------------------------------
    std::vector<int32_t> vptr(nv + 1, 0), vadj;
    {
        std::vector<std::pair<int32_t, int32_t>> pr;
        pr.reserve((size_t)nt * 12);
        for (int32_t e = 0; e < nt; ++e)
            for (int a = 0; a < 4; ++a)
                for (int b = 0; b < 4; ++b)
                    if (a != b) pr.push_back({tets[4 * e + a], tets[4 * e + b]});
        std::sort(pr.begin(), pr.end());
        pr.erase(std::unique(pr.begin(), pr.end()), pr.end());
        vadj.resize(pr.size());
        for (size_t i = 0; i < pr.size(); ++i) {
            vptr[pr[i].first + 1]++;
            vadj[i] = pr[i].second;
        }
        for (int32_t i = 0; i < nv; ++i) vptr[i + 1] += vptr[i];
    }

    // ---- separator thinning ------------------------------------------------------
    // A vertex of separator h whose neighbours (through K) lie only under one
    // child of h, or in separators at h or above, need not wait for h: it can
    // be eliminated inside that child's subtree, at the lowest node whose
    // subtree holds every such neighbour (so no two subtrees couple).  The
    // element partition leaves such vertices wherever its cut is jagged; per
    // separator, top-down, the side that takes more of them takes them all
    // (moving vertices to one side never gives another vertex a neighbour on
    // the other side, so the choice stays valid as they move).
    if (opt.thin_separators && D > 1) {
        auto in_subtree = [](int32_t a, int32_t root) {
            while (a > root) a >>= 1;
            return a == root;
        };
        auto lca = [](int32_t a, int32_t b) {
            while (a != b) {
                if (a > b) a >>= 1;
                else b >>= 1;
            }
            return a;
        };
        std::vector<std::vector<int32_t>> sep(D);
        for (int32_t v = 0; v < nv; ++v)
            if (node[v] >= 1 && node[v] < D) sep[node[v]].push_back(v);
        std::vector<uint8_t> mark(nv, 0);
        for (int32_t h = 1; h < D; ++h) {
            std::vector<int32_t>& S = sep[h];
            if (S.empty()) continue;
            std::vector<uint8_t> has(S.size(), 0);       // bit 0: under 2h, bit 1: under 2h + 1
            int32_t to_left = 0, to_right = 0;
            for (size_t i = 0; i < S.size(); ++i) {
                const int32_t v = S[i];
                for (int32_t k = vptr[v]; k < vptr[v + 1]; ++k) {
                    const int32_t w = vadj[k];
                    if (node[w] < 0 || node[w] <= h) continue;
                    if (in_subtree(node[w], 2 * h)) has[i] |= 1;
                    else if (in_subtree(node[w], 2 * h + 1)) has[i] |= 2;
                }
                if (!(has[i] & 2)) ++to_left;
                if (!(has[i] & 1)) ++to_right;
            }
            const int32_t side = (to_left >= to_right) ? 2 * h : 2 * h + 1;
            const uint8_t block = (side == 2 * h) ? 2 : 1;
            std::vector<int32_t> moved, keep;
            for (size_t i = 0; i < S.size(); ++i) (has[i] & block ? keep : moved).push_back(S[i]);
            if (moved.empty()) continue;
            // lowest node holding the neighbours already under `side` (the
            // vertices moving with v are not looked at yet)
            for (int32_t v : moved) mark[v] = 1;
            std::vector<int32_t> dest(moved.size());
            for (size_t i = 0; i < moved.size(); ++i) {
                const int32_t v = moved[i];
                int32_t n = -1;
                for (int32_t k = vptr[v]; k < vptr[v + 1]; ++k) {
                    const int32_t w = vadj[k];
                    if (node[w] < 0 || mark[w] || !in_subtree(node[w], side)) continue;
                    n = (n < 0) ? node[w] : lca(n, node[w]);
                }
                dest[i] = (n < 0) ? side : n;
            }
            for (size_t i = 0; i < moved.size(); ++i) node[moved[i]] = dest[i];
            // adjacent moved vertices must end on one root-to-leaf path: lift
            // both to their common ancestor until no pair is on two branches
            for (bool changed = true; changed;) {
                changed = false;
                for (int32_t v : moved)
                    for (int32_t k = vptr[v]; k < vptr[v + 1]; ++k) {
                        const int32_t w = vadj[k];
                        if (!mark[w]) continue;
                        const int32_t c = lca(node[v], node[w]);
                        if (c != node[v] && c != node[w]) {
                            node[v] = node[w] = c;
                            changed = true;
                        }
                    }
            }
            for (int32_t v : moved) mark[v] = 0;
            for (int32_t v : moved)
                if (node[v] < D) sep[node[v]].push_back(v);
            S.swap(keep);
        }
    }

    // Every interface tree level costs the solve a fixed latency per phase
    // (three launches), while the separators are small: the separators at odd
    // depths (1, 3, 5, ... from the root) join their parent's, halving the
    // levels, as long as the merged supernode stays within opt.merge_max_cols
    // columns (a merge replaces three sparse blocks by one denser block).
    if (D > 1 && opt.merge_max_cols > 0) {
        auto depth_of = [](int32_t h) { return 31 - __builtin_clz((uint32_t)h); };
        std::vector<int64_t> cnt(D, 0);
        for (int32_t v = 0; v < nv; ++v)
            if (node[v] >= 1 && node[v] < D) cnt[node[v]]++;
        std::vector<int32_t> into(D);
        for (int32_t h = 1; h < D; ++h) into[h] = h;
        for (int32_t h = 2; h < D; ++h) {
            if (depth_of(h) % 2 == 0) continue;
            const int32_t par = h >> 1, sib = h ^ 1;
            const int64_t merged = cnt[par] + cnt[h] + ((sib < D) ? cnt[sib] : 0);
            if (merged <= opt.merge_max_cols) into[h] = par;
        }
        for (int32_t v = 0; v < nv; ++v)
            if (node[v] >= 1 && node[v] < D) node[v] = into[node[v]];
    }

    // ---- orderings ---------------------------------------------------------------
    std::vector<std::vector<int32_t>> sub_verts(D), gam_verts(D);   // gam_verts[h], h in [1, D)
    for (int32_t v = 0; v < nv; ++v) {
        if (node[v] < 0) continue;
        if (node[v] >= D) sub_verts[node[v] - D].push_back(v);
        else gam_verts[node[v]].push_back(v);
    }
    std::vector<std::vector<NDNode>> ndt(D);
    std::vector<int32_t> ndroot(D, -1);
#pragma omp parallel
    {
        NDScratch sc;
        sc.mark.assign(nv, 0);
        sc.level.assign(nv, 0);
#pragma omp for schedule(dynamic, 1)
        for (int32_t d = 0; d < D; ++d)
            if (!sub_verts[d].empty())
                ndroot[d] = nd_build(sub_verts[d], leaf_max, vptr, vadj, sc, ndt[d]);
    }

    // supernodes in global postorder
    std::vector<Supernode>& SN = P.sn;
    std::vector<int32_t> order;   // internal id -> user vertex (free part)
    order.reserve(nv);
    P.sub_off.assign(D + 1, 0);
    std::vector<int32_t> sub_root_sn(D, -1);
    for (int32_t d = 0; d < D; ++d) {
        P.sub_off[d] = (int32_t)order.size();
        if (ndroot[d] < 0) continue;
        // iterative postorder of the ND tree; returns supernode id of each ND node
        std::vector<NDNode>& T = ndt[d];
        std::vector<int32_t> snid(T.size(), -1), snid_last(T.size(), -1);
        std::vector<std::pair<int32_t, int>> st;
        st.push_back({ndroot[d], 0});
        while (!st.empty()) {
            auto& top = st.back();
            int32_t u = top.first;
            if (top.second == 0) {
                top.second = 1;
                if (T[u].left >= 0) st.push_back({T[u].left, 0});
            } else if (top.second == 1) {
                top.second = 2;
                if (T[u].right >= 0) st.push_back({T[u].right, 0});
            } else {
                st.pop_back();
                if (!T[u].verts.empty()) {
                    // pieces of at most kMaxInteriorCols columns, chained: each
                    // piece's parent is the next one (a separator's diagonal
                    // block is dense, so every piece's rows include the later ones)
                    const int32_t nvts = (int32_t)T[u].verts.size();
                    const int32_t npc = (nvts + kMaxInteriorCols - 1) / kMaxInteriorCols;
                    snid[u] = (int32_t)SN.size();
                    for (int32_t pc = 0; pc < npc; ++pc) {
                        const int32_t a0 = pc * nvts / npc, a1 = (pc + 1) * nvts / npc;
                        Supernode s;
                        s.col0 = (int32_t)order.size();
                        s.n = a1 - a0;
                        s.sub = d;
                        for (int32_t k = a0; k < a1; ++k) order.push_back(T[u].verts[k]);
                        if (pc + 1 < npc) s.parent = (int32_t)SN.size() + 1;
                        SN.push_back(std::move(s));
                    }
                    snid_last[u] = (int32_t)SN.size() - 1;
                }
            }
        }
        // parents inside the subdomain: nearest non-empty ND ancestor
        std::vector<int32_t> ndpar(T.size(), -1);
        for (size_t u = 0; u < T.size(); ++u) {
            if (T[u].left >= 0) ndpar[T[u].left] = (int32_t)u;
            if (T[u].right >= 0) ndpar[T[u].right] = (int32_t)u;
        }
        for (size_t u = 0; u < T.size(); ++u) {
            if (snid[u] < 0) continue;
            int32_t a = ndpar[u];
            while (a >= 0 && snid[a] < 0) a = ndpar[a];
            // the last piece hangs below the first piece of the nearest non-empty ancestor
            SN[snid_last[u]].parent = (a >= 0) ? snid[a] : -2;   // -2: attach to interface later
        }
    }
    P.sub_off[D] = (int32_t)order.size();
    P.n_int = (int32_t)order.size();
    // interface supernodes in heap postorder
    std::vector<int32_t> heap_sn(2 * D, -1);
    {
        std::vector<std::pair<int32_t, int>> st;
        if (D > 1) st.push_back({1, 0});
        while (!st.empty()) {
            auto& top = st.back();
            int32_t h = top.first;
            if (top.second == 0) {
                top.second = 1;
                if (2 * h < D) st.push_back({2 * h, 0});
            } else if (top.second == 1) {
                top.second = 2;
                if (2 * h + 1 < D) st.push_back({2 * h + 1, 0});
            } else {
                st.pop_back();
                auto& gv = gam_verts[h];
                if (!gv.empty()) {
                    std::sort(gv.begin(), gv.end());
                    Supernode s;
                    s.col0 = (int32_t)order.size();
                    s.n = (int32_t)gv.size();
                    s.sub = -1;
                    for (int32_t v : gv) order.push_back(v);
                    heap_sn[h] = (int32_t)SN.size();
                    SN.push_back(std::move(s));
                }
            }
        }
    }
    P.n_free = (int32_t)order.size();
    P.n_gamma = P.n_free - P.n_int;
    auto heap_parent_sn = [&](int32_t h) {
        h >>= 1;
        while (h >= 1 && heap_sn[h] < 0) h >>= 1;
        return h >= 1 ? heap_sn[h] : -1;
    };
    for (int32_t h = 1; h < D; ++h)
        if (heap_sn[h] >= 0) SN[heap_sn[h]].parent = heap_parent_sn(h);
    for (auto& s : SN)
        if (s.parent == -2) s.parent = heap_parent_sn(D + s.sub);
    for (int32_t t = 0; t < (int32_t)SN.size(); ++t)
        if (SN[t].parent >= 0) SN[SN[t].parent].children.push_back(t);
    // heights
    for (int32_t t = 0; t < (int32_t)SN.size(); ++t) {
        Supernode& s = SN[t];
        if (s.sub >= 0) {
            int32_t h = 0;
            for (int32_t c : s.children) h = std::max(h, SN[c].height + 1);
            s.height = h;
        } else {
            int32_t h = 0;
            for (int32_t c : s.children)
                if (SN[c].sub < 0) h = std::max(h, SN[c].clevel + 1);
            s.clevel = h;
            P.n_clevels = std::max(P.n_clevels, h + 1);
        }
    }

    // internal numbering: free in `order`, then pinned
    P.perm = order;
    for (int32_t v = 0; v < nv; ++v)
        if (pinned[v]) P.perm.push_back(v);
    if ((int32_t)P.perm.size() != nv) {
        msg = "vertex numbering failed";
        return EINVAL_;
    }
    P.iperm.assign(nv, 0);
    for (int32_t i = 0; i < nv; ++i) P.iperm[P.perm[i]] = i;
    P.X_int.resize((size_t)nv * 3);
    P.mass_int.resize(nv);
    for (int32_t i = 0; i < nv; ++i) {
        int32_t u = P.perm[i];
        for (int c = 0; c < 3; ++c) P.X_int[3 * i + c] = X[3 * u + c];
        P.mass_int[i] = mass[u];
    }

    // ---- elements: sorted by subdomain, SoA geometry -------------------------
    P.elem_perm.resize(nt);
    std::iota(P.elem_perm.begin(), P.elem_perm.end(), 0);
    std::stable_sort(P.elem_perm.begin(), P.elem_perm.end(),
                     [&](int32_t a, int32_t b) { return part[a] < part[b]; });
    P.tet_soa.resize((size_t)nt * 4);
    P.trec.assign((size_t)nt * 16, 0.0f);
    std::vector<double> Vol(nt), Gd((size_t)nt * 9);
    for (int32_t e = 0; e < nt; ++e) {
        int32_t u = P.elem_perm[e];
        const int32_t* t = tets + 4 * u;
        double Dm[9], G[9];
        tet_dm(X, t, Dm);
        double det = det3(Dm);
        inv3(Dm, det, G);
        Vol[e] = det / 6.0;
        float* rec = &P.trec[(size_t)e * 16];
        for (int c = 0; c < 4; ++c) {
            P.tet_soa[(size_t)c * nt + e] = P.iperm[t[c]];
            int32_t id = P.iperm[t[c]];
            std::memcpy(&rec[c], &id, 4);
        }
        for (int k = 0; k < 9; ++k) {
            rec[4 + k] = (float)G[k];
            Gd[(size_t)e * 9 + k] = G[k];
        }
        rec[13] = (float)(Vol[e] * gamma_s[u]);
        rec[14] = (float)(Vol[e] * gamma_v[u]);
        rec[15] = (float)Vol[e];
    }

    // ---- scatter: per-block reduction of corner forces ----------------------------
    {
        const int32_t nblocks = (nt + kLocalBlock - 1) / kLocalBlock;
        P.lpos.assign((size_t)4 * nt, 0xFFFF);
        P.blk_part.assign(nblocks + 1, 0);
        P.part_pack.clear();
        std::vector<std::vector<int32_t>> vparts(P.n_free);
        std::vector<std::pair<int32_t, int32_t>> inc;   // (vertex, local corner slot t*4 + c)
        for (int32_t b = 0; b < nblocks; ++b) {
            P.blk_part[b] = (int32_t)P.part_pack.size();
            const int32_t e0 = b * kLocalBlock, e1 = std::min(nt, e0 + kLocalBlock);
            inc.clear();
            for (int32_t e = e0; e < e1; ++e)
                for (int32_t c = 0; c < 4; ++c) {
                    int32_t a = P.tet_soa[(size_t)c * nt + e];
                    if (a < P.n_free) inc.push_back({a, (e - e0) * 4 + c});
                }
            std::sort(inc.begin(), inc.end());
            for (size_t k = 0; k < inc.size();) {
                size_t k1 = k;
                while (k1 < inc.size() && inc[k1].first == inc[k].first) ++k1;
                const int32_t pidx = (int32_t)P.part_pack.size();
                P.part_pack.push_back(((int32_t)k << 16) | (int32_t)(k1 - k));
                vparts[inc[k].first].push_back(pidx);
                for (size_t q = k; q < k1; ++q) {
                    const int32_t slot = inc[q].second;
                    P.lpos[(size_t)(e0 + slot / 4) * 4 + slot % 4] = (uint16_t)q;
                }
                k = k1;
            }
        }
        P.blk_part[nblocks] = (int32_t)P.part_pack.size();
        P.vpart_ptr.assign(P.n_free + 1, 0);
        P.vpart.clear();
        for (int32_t a = 0; a < P.n_free; ++a) {
            P.vpart.insert(P.vpart.end(), vparts[a].begin(), vparts[a].end());
            P.vpart_ptr[a + 1] = (int32_t)P.vpart.size();
        }
    }

    // ---- FP64 matrix on free unknowns (internal order) ------------------------------
    const int32_t nf = P.n_free;
    assemble_matrix(P, Vol, Gd, gamma_s, gamma_v, dt);

    // ---- symbolic: rows below each supernode --------------------------------------
    const int32_t nsn = (int32_t)SN.size();
    auto symbolic = [&](int32_t t, std::vector<int32_t>& buf) {
        Supernode& s = SN[t];
        int32_t last = s.col0 + s.n - 1;
        buf.clear();
        for (int32_t c : s.children)
            for (int32_t r : SN[c].rows)
                if (r > last) buf.push_back(r);
        for (int32_t j = s.col0; j <= last; ++j)
            for (int32_t k = P.K_ptr[j]; k < P.K_ptr[j + 1]; ++k)
                if (P.K_col[k] > last) buf.push_back(P.K_col[k]);
        std::sort(buf.begin(), buf.end());
        buf.erase(std::unique(buf.begin(), buf.end()), buf.end());
        s.rows = buf;
    };
    {
        // interior supernodes: independent per subdomain (postorder inside)
        std::vector<int32_t> sub_first(D + 1, nsn);
        for (int32_t t = nsn - 1; t >= 0; --t)
            if (SN[t].sub >= 0) sub_first[SN[t].sub] = t;
#pragma omp parallel
        {
            std::vector<int32_t> buf;
#pragma omp for schedule(dynamic, 1)
            for (int32_t d = 0; d < D; ++d)
                for (int32_t t = 0; t < nsn; ++t) {
                    if (SN[t].sub != d) continue;
                    symbolic(t, buf);
                }
        }
        std::vector<int32_t> buf;
        for (int32_t t = 0; t < nsn; ++t)
            if (SN[t].sub < 0) symbolic(t, buf);
        (void)sub_first;
    }
    // value offsets.  Per supernode t with inverted diagonal block Ti = L_tt^{-1}
    // and rows below B (m x n), the solve uses W_B = B Ti:
    //   forward   [z_t; c_t] = [Ti; W_B] r'_t      (c_t: contributions to the rows below)
    //   backward  d_t = Ti^T z_t - W_B^T d_{R_t}
    // Wf (row-major rows of [Ti; W_B]) and Wb (columns of [Ti; -W_B], each from its
    // diagonal down) are stored, tri + m n values each.
    int64_t fo = 0, dof = 0;
    for (int32_t t = 0; t < nsn; ++t) {
        Supernode& s = SN[t];
        int64_t n = s.n, m = (int64_t)s.rows.size();
        int64_t blk = n * (n + 1) / 2 + m * n;
        int64_t& o = (s.sub >= 0) ? fo : dof;
        s.wf_off = o;
        o += blk;
        s.wb_off = o;
        o += blk;
        if (s.sub >= 0) P.nnz_int += blk;
        else P.nnz_coarse += blk;
    }
    if (dof >= ((int64_t)1 << 31)) {
        msg = "interface factor too large for 32-bit offsets";
        return ENOMEM_;
    }
    std::vector<double> ivd;
    try {
        ivd.assign(fo, 0.0);
        P.dvals.assign(dof, 0.0);
    } catch (...) {
        msg = "host allocation of the factor failed";
        return ENOMEM_;
    }

    // ---- numeric: multifrontal FP64 --------------------------------------------------
    P.n_ivd = fo;
    P.iface_on_device = opt.iface_on_device;
    {
        const int rc = factor_numeric(P, ivd, msg);
        if (rc != OK) return rc;
    }

    // ---- contribution slots ------------------------------------------------------------
    // Row p of supernode t contributes c_t[p] to row R_t[p].  Interior rows of an
    // interior supernode get a slot in its subdomain's LDS buffer, interface rows of
    // an interior supernode a global FP32 slot, rows of an interface supernode a
    // global FP64 slot.  Each receiving row sums its slots in (t, p) order.
    std::vector<std::vector<int32_t>> pull_i(nf), pull_f(nf), pull_d(nf);
    std::vector<int32_t> cint_used(D, 0);
    int32_t ncgf = 0, ncgd = 0;
    for (int32_t t = 0; t < nsn; ++t) {
        Supernode& S = SN[t];
        const int32_t m = (int32_t)S.rows.size();
        int32_t mi = 0;
        while (mi < m && S.rows[mi] < P.n_int) ++mi;
        S.m_int = mi;
        if (S.sub >= 0) {
            S.cint0 = cint_used[S.sub];
            cint_used[S.sub] += mi;
            S.cg0 = ncgf;
            ncgf += m - mi;
            for (int32_t p = 0; p < mi; ++p) pull_i[S.rows[p]].push_back(S.cint0 + p);
            for (int32_t p = mi; p < m; ++p) pull_f[S.rows[p]].push_back(S.cg0 + p - mi);
        } else {
            S.cg0 = ncgd;
            ncgd += m;
            for (int32_t p = 0; p < m; ++p) pull_d[S.rows[p]].push_back(S.cg0 + p);
        }
    }
    P.n_cgf = ncgf;
    P.n_cgd = ncgd;
    // Slot numbers grouped by the receiving row: each interface row's FP32 and
    // FP64 slots are contiguous, in its summation order, so an interface
    // PULLSUM reads two runs and needs no slot list.
    std::vector<int32_t> fslot(ncgf, -1), dslot(ncgd, -1), fbase(nf, 0), dbase(nf, 0);
    {
        int32_t nfs = 0, nds = 0;
        for (int32_t r = P.n_int; r < nf; ++r) {
            fbase[r] = nfs;
            for (int32_t o : pull_f[r]) fslot[o] = nfs++;
            dbase[r] = nds;
            for (int32_t o : pull_d[r]) dslot[o] = nds++;
        }
        if (nfs != ncgf || nds != ncgd) {
            msg = "contribution slots not all received by interface rows";
            return EINVAL_;
        }
    }
    P.max_cint = 0;
    for (int32_t d = 0; d < D; ++d) P.max_cint = std::max(P.max_cint, cint_used[d]);

    // ---- interior programs: LDS chunks ---------------------------------------------
    // A chunk is [ntasks x 8 int32 task descriptors][data], all as 32-bit words
    // (ints bit-cast into the float array); data offsets are relative to the data
    // start.  Local vector ids: [0, n_loc) interior rows, [n_loc, n_loc + nb) the
    // subdomain's boundary rows staged from the interface solution.
    P.chunk_floats = chunk_floats;
    P.bnd_off.assign(D + 1, 0);
    P.bnd.clear();
    std::vector<std::vector<int32_t>> sub_sn(D);
    for (int32_t t = 0; t < nsn; ++t)
        if (SN[t].sub >= 0) sub_sn[SN[t].sub].push_back(t);
    for (int32_t d = 0; d < D; ++d) {
        P.bnd_off[d] = (int32_t)P.bnd.size();
        std::vector<int32_t> bl;
        for (int32_t t : sub_sn[d])
            for (int32_t r : SN[t].rows)
                if (r >= P.n_int) bl.push_back(r);
        std::sort(bl.begin(), bl.end());
        bl.erase(std::unique(bl.begin(), bl.end()), bl.end());
        P.bnd.insert(P.bnd.end(), bl.begin(), bl.end());
        P.max_nb = std::max(P.max_nb, (int32_t)bl.size());
        P.max_sub_n = std::max(P.max_sub_n, P.sub_off[d + 1] - P.sub_off[d]);
    }
    P.bnd_off[D] = (int32_t)P.bnd.size();
    std::vector<int32_t> bpos(nf, -1);
    auto as_f = [](int32_t v) {
        float f;
        std::memcpy(&f, &v, 4);
        return f;
    };
    // Chunk layouts (32-bit words; ints bit-cast into the float array):
    //   PULLSUM: ntasks x {row, list offset, count, 0}, then the slot lists
    //   GEMV:    ntasks x {col0, n, m, m_int, cint0, slot list offset, value
    //            offset, row0}, then per supernode its column-major block
    //            (column k: rows k..n+m-1) and the FP32 slots of its interface rows
    //   BGEMV:   ntasks x {col0, n, m, value offset, gather offset, col0 of the
    //            block, 0, 0}, then gather lists and row-major blocks
    // Descriptors are 8 words (PULLSUM uses 4); data offsets are relative to the
    // data start, which is desc_words * ntasks.
    struct Builder {
        int32_t kind = 0;
        std::vector<int32_t> desc;
        std::vector<float> data;
        std::vector<int32_t> src;   // per data word: its FP64 interior value, or -1
        void word(float w) {
            data.push_back(w);
            src.push_back(-1);
        }
        void value(const std::vector<double>& v, int64_t o) {
            data.push_back((float)v[o]);
            src.push_back((int32_t)o);
        }
    } cb;
    bool too_big = false;
    auto dwords = [](int32_t kind) { return kind == PULLSUM ? 4 : 8; };
    auto flush = [&]() {
        const int32_t nt_ = (int32_t)cb.desc.size() / dwords(cb.kind);
        if (nt_ == 0) return;
        while (P.ivals.size() % 4) {
            P.ivals.push_back(0.0f);
            P.ival_src.push_back(-1);
        }
        Chunk c;
        c.kind = cb.kind;
        c.ntasks = nt_;
        c.v0 = (int32_t)P.ivals.size();
        for (int32_t v : cb.desc) P.ivals.push_back(as_f(v));
        P.ival_src.insert(P.ival_src.end(), cb.desc.size(), -1);
        P.ivals.insert(P.ivals.end(), cb.data.begin(), cb.data.end());
        P.ival_src.insert(P.ival_src.end(), cb.src.begin(), cb.src.end());
        c.nv = (int32_t)P.ivals.size() - c.v0;
        c.pad[0] = c.pad[1] = c.pad[2] = c.pad[3] = 0;
        if (c.nv > chunk_floats) too_big = true;
        P.chunks.push_back(c);
        cb.desc.clear();
        cb.data.clear();
        cb.src.clear();
    };
    auto room = [&](int32_t need_words) {
        return (int32_t)(cb.desc.size() + cb.data.size()) + need_words <= chunk_floats || cb.desc.empty();
    };
    auto start_phase = [&](int32_t kind) {
        flush();
        cb.kind = kind;
    };
    P.ivals.clear();
    P.ival_src.clear();
    P.chunks.clear();
    P.sub_fwd_ch.assign(D + 1, 0);
    P.sub_bwd_ch.assign(D + 1, 0);
    for (int32_t d = 0; d < D; ++d) {
        P.sub_fwd_ch[d] = (int32_t)P.chunks.size();
        const int32_t base = P.sub_off[d];
        int32_t H = -1;
        for (int32_t t : sub_sn[d]) H = std::max(H, SN[t].height);
        for (int32_t h = 0; h <= H; ++h) {
            start_phase(PULLSUM);
            for (int32_t t : sub_sn[d]) {
                if (SN[t].height != h) continue;
                for (int32_t a = 0; a < SN[t].n; ++a) {
                    const auto& L = pull_i[SN[t].col0 + a];
                    if (L.empty()) continue;
                    if (!room(4 + (int32_t)L.size())) flush();
                    int32_t off = (int32_t)cb.data.size();
                    for (int32_t sl : L) cb.word(as_f(sl));
                    int32_t dsc[4] = {SN[t].col0 + a - base, off, (int32_t)L.size(), 0};
                    cb.desc.insert(cb.desc.end(), dsc, dsc + 4);
                }
            }
            start_phase(GEMV);
            for (int32_t t : sub_sn[d]) {
                if (SN[t].height != h) continue;
                const Supernode& S = SN[t];
                const int32_t n = S.n, m = (int32_t)S.rows.size();
                const int32_t blk = n * (n + 1) / 2 + m * n;
                const int32_t nblk_rows = (n + m + 63) / 64;
                if (!room(8 * nblk_rows + blk + (m - S.m_int))) flush();
                const int32_t off = (int32_t)cb.data.size();
                for (int32_t q = 0; q < blk; ++q) cb.value(ivd, S.wb_off + q);
                const int32_t soff = (int32_t)cb.data.size();   // FP32 slots of the interface rows
                for (int32_t p = S.m_int; p < m; ++p) cb.word(as_f(fslot[S.cg0 + p - S.m_int]));
                for (int32_t rb = 0; rb < nblk_rows; ++rb) {
                    int32_t dsc[8] = {S.col0 - base, n, m, S.m_int, S.cint0, soff, off, 64 * rb};
                    cb.desc.insert(cb.desc.end(), dsc, dsc + 8);
                }
            }
            flush();
        }
        P.max_sub_phases = std::max(P.max_sub_phases, 2 * (H + 1));
    }
    P.sub_fwd_ch[D] = (int32_t)P.chunks.size();
    for (int32_t d = 0; d < D; ++d) {
        P.sub_bwd_ch[d] = (int32_t)P.chunks.size();
        const int32_t base = P.sub_off[d];
        const int32_t nloc = P.sub_off[d + 1] - base;
        for (int32_t k = P.bnd_off[d]; k < P.bnd_off[d + 1]; ++k) bpos[P.bnd[k]] = nloc + (k - P.bnd_off[d]);
        int32_t H = -1;
        for (int32_t t : sub_sn[d]) H = std::max(H, SN[t].height);
        for (int32_t h = H; h >= 0; --h) {
            start_phase(BGEMV);
            for (int32_t t : sub_sn[d]) {
                if (SN[t].height != h) continue;
                const Supernode& S = SN[t];
                const int32_t n = S.n, m = (int32_t)S.rows.size();
                const int32_t blk = n * (n + 1) / 2 + m * n;
                const int32_t nblk_cols = (n + 63) / 64;
                if (!room(8 * nblk_cols + m + blk)) flush();
                const int32_t goff = (int32_t)cb.data.size();
                for (int32_t r : S.rows) cb.word(as_f(r < P.n_int ? r - base : bpos[r]));
                const int32_t off = (int32_t)cb.data.size();
                for (int32_t q = 0; q < blk; ++q) cb.value(ivd, S.wf_off + q);
                for (int32_t cbk = 0; cbk < nblk_cols; ++cbk) {
                    int32_t dsc[8] = {S.col0 - base, n, m, off, goff, 64 * cbk, 0, 0};
                    cb.desc.insert(cb.desc.end(), dsc, dsc + 8);
                }
            }
            flush();
        }
    }
    P.sub_bwd_ch[D] = (int32_t)P.chunks.size();
    while (P.ivals.size() % 4) {
        P.ivals.push_back(0.0f);
        P.ival_src.push_back(-1);
    }
    if (too_big) {
        msg = "an interior supernode's solve block does not fit one LDS chunk";
        return EINVAL_;
    }

    // ---- interface programs: one launch per phase ------------------------------------
    P.ctasks.clear();
    P.cslots.clear();
    P.cgidx.clear();
    P.cfwd.clear();
    P.cbwd.clear();
    // lanes per interface task by the phase's mean task length
    const int64_t g32_min = opt.lanes32_min, g64_min = opt.lanes64_min;
    auto open_cphase = [&](int32_t kind) {
        CPhase ph;
        ph.kind = kind;
        ph.task0 = (int32_t)P.ctasks.size();
        ph.ntasks = 0;
        ph.group = 16;
        return ph;
    };
    auto close_cphase = [&](CPhase ph, int64_t total_len, std::vector<CPhase>& lst) {
        ph.ntasks = (int32_t)P.ctasks.size() - ph.task0;
        if (ph.ntasks == 0) return;
        const int64_t avg = total_len / ph.ntasks;
        ph.group = (avg >= g64_min) ? 64 : (avg >= g32_min) ? 32 : 16;
        lst.push_back(ph);
    };
    std::vector<int32_t> cg_goff(nsn, -1);
    for (int32_t t = 0; t < nsn; ++t)
        if (SN[t].sub < 0) {
            cg_goff[t] = (int32_t)P.cgidx.size();
            for (int32_t r : SN[t].rows) P.cgidx.push_back(r - P.n_int);
        }
    for (int32_t l = 0; l < P.n_clevels; ++l) {
        CPhase ph = open_cphase(PULLSUM);
        int64_t tl = 0;
        for (int32_t t = 0; t < nsn; ++t) {
            if (SN[t].sub >= 0 || SN[t].clevel != l) continue;
            for (int32_t a = 0; a < SN[t].n; ++a) {
                const int32_t r = SN[t].col0 + a;
                CTask c{};
                c.a[0] = r - P.n_int;
                c.a[1] = fbase[r];
                c.a[2] = (int32_t)pull_f[r].size();
                c.a[3] = dbase[r];
                c.a[4] = (int32_t)pull_d[r].size();
                tl += c.a[2] + c.a[4];
                P.ctasks.push_back(c);
            }
        }
        close_cphase(ph, tl, P.cfwd);
        ph = open_cphase(GEMV);
        tl = 0;
        for (int32_t t = 0; t < nsn; ++t) {
            if (SN[t].sub >= 0 || SN[t].clevel != l) continue;
            const Supernode& S = SN[t];
            const int32_t n = S.n, m = (int32_t)S.rows.size();
            const int64_t tri = (int64_t)n * (n + 1) / 2;
            if (m == 0) {
                // a root: rows of A = Ti^T Ti straight into the solution
                for (int32_t i = 0; i < n; ++i) {
                    CTask c{};
                    c.a[0] = 2;
                    c.a[1] = S.col0 - P.n_int + i;
                    c.a[2] = (int32_t)(S.wf_off + (int64_t)i * n);
                    c.a[3] = n;
                    c.a[4] = S.col0 - P.n_int;
                    tl += n;
                    P.ctasks.push_back(c);
                }
                continue;
            }
            for (int32_t i = 0; i < n + m; ++i) {
                CTask c{};
                c.a[0] = (i < n) ? 0 : 1;
                c.a[1] = (i < n) ? S.col0 - P.n_int + i : dslot[S.cg0 + (i - n)];
                c.a[2] = (int32_t)(S.wf_off + ((i < n) ? (int64_t)i * (i + 1) / 2 : tri + (int64_t)(i - n) * n));
                c.a[3] = (i < n) ? i + 1 : n;
                c.a[4] = S.col0 - P.n_int;
                tl += c.a[3];
                P.ctasks.push_back(c);
            }
        }
        close_cphase(ph, tl, P.cfwd);
    }
    for (int32_t l = P.n_clevels - 1; l >= 0; --l) {
        CPhase ph = open_cphase(BGEMV);
        int64_t tl = 0;
        for (int32_t t = 0; t < nsn; ++t) {
            if (SN[t].sub >= 0 || SN[t].clevel != l) continue;
            const Supernode& S = SN[t];
            const int32_t n = S.n, m = (int32_t)S.rows.size();
            if (m == 0) continue;   // a root was solved whole in the forward pass
            for (int32_t k = 0; k < n; ++k) {
                CTask c{};
                c.a[0] = S.col0 - P.n_int + k;
                c.a[1] = (int32_t)(S.wb_off + (int64_t)k * (n + m) - (int64_t)k * (k - 1) / 2);
                c.a[2] = n - k;
                c.a[3] = S.col0 - P.n_int + k;
                c.a[4] = m;
                c.a[5] = cg_goff[t];
                tl += n - k + m;
                P.ctasks.push_back(c);
            }
        }
        close_cphase(ph, tl, P.cbwd);
    }
    P.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t_start).count();
    return OK;
}

int refactor_plan(Plan& P, const double* X, const int32_t* tets, const double* gamma_s, const double* gamma_v,
                  std::string& msg) {
    auto t_start = std::chrono::steady_clock::now();
    const int32_t nt = P.nt;
    std::vector<double> Vol(nt), Gd((size_t)nt * 9);
    for (int32_t e = 0; e < nt; ++e) {
        const int32_t u = P.elem_perm[e];
        double Dm[9], G[9];
        tet_dm(X, tets + 4 * u, Dm);
        const double det = det3(Dm);
        inv3(Dm, det, G);
        Vol[e] = det / 6.0;
        for (int k = 0; k < 9; ++k) Gd[(size_t)e * 9 + k] = G[k];
        P.trec[(size_t)e * 16 + 13] = (float)(Vol[e] * gamma_s[u]);
        P.trec[(size_t)e * 16 + 14] = (float)(Vol[e] * gamma_v[u]);
    }
    assemble_matrix(P, Vol, Gd, gamma_s, gamma_v, P.dt);
    std::vector<double> ivd;
    try {
        ivd.assign(P.n_ivd, 0.0);
    } catch (...) {
        msg = "host allocation of the factor failed";
        return ENOMEM_;
    }
    std::fill(P.dvals.begin(), P.dvals.end(), 0.0);
    const int rc = factor_numeric(P, ivd, msg);
    if (rc != OK) return rc;
    for (size_t k = 0; k < P.ivals.size(); ++k)
        if (P.ival_src[k] >= 0) P.ivals[k] = (float)ivd[P.ival_src[k]];
    P.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t_start).count();
    return OK;
}

}  // namespace vh
