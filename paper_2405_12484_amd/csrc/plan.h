// Host-side plan of one garment: everything the device path needs, built in
// FP64 on the host once per material (the global matrix of Sec. 7.1 is
// constant, so it is factored once; Sec. 7.2).
#pragma once

#include <cstdint>
#include <string>
#include <vector>

namespace vh {

// Supernode of the nested-dissection tree: contiguous columns [col0, col0+n)
// of the permuted free unknowns, with the rows below its diagonal block
// (rows[], ascending, all inside ancestor supernodes).
struct Supernode {
    int32_t col0 = 0, n = 0;
    int32_t parent = -1;
    int32_t sub = -1;        // owning subdomain, -1 for interface supernodes
    int32_t height = 0;      // 0 at leaves; interior: within the subdomain tree
    int32_t clevel = -1;     // interface supernodes: level in the interface tree
    std::vector<int32_t> children;
    std::vector<int32_t> rows;
    // offsets into the value arrays (float for interior, double for interface)
    int64_t tinv_off = 0, tinvT_off = 0, b_off = 0, bT_off = 0, rows_off = 0;
};

// One dot-product term of a solve task: sum_k vals[voff + k] * x[xoff + k]
// (contiguous) or x[gidx[xoff + k]] (gathered), k < len.
struct Seg {
    int32_t voff;   // offset in the value array (elements); values may exceed 2^31 -> split
    int32_t len;
    int32_t xoff;
    int32_t kind;   // 0: double values / double x (interface), 1: float / float (interior)
};
struct Task {
    int32_t out;      // output slot
    int32_t seg0, seg1;
    int32_t pad;
};
struct Phase {
    int32_t kind;     // 0 fwd pull, 1 fwd tinv, 2 bwd pull, 3 bwd tinv
    int32_t task0, task1;
    int32_t pad;
};

enum PhaseKind { FWD_PULL = 0, FWD_TINV = 1, BWD_PULL = 2, BWD_TINV = 3 };

// A piece of an interior phase whose values (and gather indices) are
// contiguous in Plan::ivals, so one workgroup can stage it in LDS with one
// coalesced copy.  Segment voff/xoff of its tasks are relative to v0.
struct Chunk {
    int32_t kind;
    int32_t task0, task1;
    int32_t v0, nv;       // [v0, v0 + nv) in ivals, v0 % 4 == 0
    int32_t pad[3];
};

struct Plan {
    // sizes
    int32_t nv = 0, nt = 0, n_free = 0, n_int = 0, n_gamma = 0, D = 1;
    double dt = 0, gravity[3] = {0, 0, 0};
    int32_t pd_iters = 10, refine_steps = 0;

    // vertex numbering: internal id -> user id and back.  Internal ids:
    // [0, n_int) subdomain interiors (subdomain-major, nested-dissection
    // order), [n_int, n_free) interface, [n_free, nv) pinned.
    std::vector<int32_t> perm, iperm;
    std::vector<int32_t> sub_off;         // D+1 interior ranges
    std::vector<double> X_int;            // nv*3 rest positions, internal order
    std::vector<double> mass_int;         // nv
    std::vector<uint8_t> pinned_user;     // nv, user order

    // elements in internal order (sorted by subdomain), SoA
    std::vector<int32_t> elem_perm;       // internal element -> user element
    std::vector<int32_t> tet_soa;         // 4*nt internal vertex ids
    std::vector<float> ginv_soa;          // 9*nt, Dm^{-1} row-major per tet
    std::vector<float> w_soa;             // 2*nt  (V gs, V gv)

    // scatter: free vertex -> incident (corner, element) slots c*nt + e
    std::vector<int32_t> inc_ptr, inc_slot;

    // FP64 free-free matrix in internal order (CSR) for refinement residuals
    std::vector<int32_t> K_ptr, K_col;
    std::vector<double> K_val;

    // factor
    std::vector<Supernode> sn;
    std::vector<float> fvals;             // interior factor blocks
    std::vector<double> dvals;            // interface factor blocks
    std::vector<int32_t> gidx;            // gather indices (rows lists)
    int64_t nnz_int = 0, nnz_coarse = 0;

    // solve programs
    std::vector<Seg> segs;
    std::vector<Task> tasks;
    std::vector<Phase> phases;
    std::vector<int32_t> sub_fwd_ph, sub_bwd_ph;   // D+1 ranges into phases (per subdomain)
    // interior programs as LDS chunks (values and gather indices packed)
    std::vector<Chunk> chunks;
    std::vector<int32_t> sub_fwd_ch, sub_bwd_ch;   // D+1 ranges into chunks
    std::vector<float> ivals;                      // packed interior values
    std::vector<int32_t> bnd, bnd_off;             // per subdomain: interface rows it touches
    int32_t max_nb = 0, chunk_floats = 0;
    std::vector<int32_t> coarse_fwd_ph, coarse_bwd_ph;  // ranges of phases, one launch each
    int32_t max_sub_phases = 0, max_sub_n = 0, n_clevels = 0;

    double seconds = 0;
};

// Build a plan; returns 0 or a negative VH_E* code with msg set.
int build_plan(const double* X, int32_t nv, const int32_t* tets, int32_t nt,
               const double* gamma_s, const double* gamma_v, const double* mass,
               const uint8_t* pinned, const double* gravity, double dt, int32_t pd_iters,
               int32_t n_subdomains, int32_t refine_steps, int32_t leaf_max,
               int32_t chunk_floats, Plan& plan, std::string& msg);

// Rest-shape checks used at mesh creation: every tet has positive volume.
int check_mesh(const double* X, int32_t nv, const int32_t* tets, int32_t nt, std::string& msg);

}  // namespace vh
