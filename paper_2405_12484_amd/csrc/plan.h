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
    int32_t m_int = 0;       // rows below that are interior rows (they come first)
    int32_t cint0 = 0;       // first LDS contribution slot (interior supernodes)
    int32_t cg0 = 0;         // first global contribution slot
    // offsets of the forward / backward value blocks (float staging for interior,
    // Plan::dvals for interface supernodes)
    int64_t wf_off = 0, wb_off = 0;
};

// Solve task kinds.  PULLSUM: r'_row = r_row - sum of contribution slots;
// GEMV: one row of [z; c] = [Ti; B Ti] r'; BGEMV: one column of
// d = Ti^T z - (B Ti)^T d_rows.
enum TaskKind { PULLSUM = 0, GEMV = 1, BGEMV = 2 };

// A piece of an interior phase stored contiguously in Plan::ivals:
// [ntasks x 8 int32 descriptors][data], one coalesced copy into LDS.
//   PULLSUM: {row, data offset of the slot list, count}
//   GEMV:    {dest (0 z, 1 LDS slot, 2 global FP32 slot), index, data offset, len, x offset}
//   BGEMV:   {out, data offset, len1, z offset, len2, data offset of the gather list}
struct Chunk {
    int32_t kind;
    int32_t ntasks;
    int32_t v0, nv;       // [v0, v0 + nv) in ivals, v0 % 4 == 0
    int32_t pad[4];
};

// Interface task (global memory, FP64 values):
//   PULLSUM: {row, first FP32 slot, count, first FP64 slot, count} (a row's slots are contiguous)
//   GEMV:    {dest (0 z, 1 FP64 slot, 2 solution d), index, value offset, len, x offset}
//            (dest 2: a root supernode, whose rows of A = Ti^T Ti give d at once)
//   BGEMV:   {out, value offset, len1, z offset, len2, gather list offset}
struct CTask {
    int32_t a[8];
};
struct CPhase {
    int32_t kind, task0, ntasks, group;   // group: lanes per task (16 or 64)
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

    // elements in internal order (sorted by subdomain)
    std::vector<int32_t> elem_perm;       // internal element -> user element
    std::vector<int32_t> tet_soa;         // 4*nt internal vertex ids (host use)
    // one 64-byte record per tet: 4 vertex ids, Dm^{-1} (9, row-major), V gs, V gv, 0
    std::vector<float> trec;              // 16*nt 32-bit words
    // scatter, reduced per block of kLocalBlock tets: each corner force goes to
    // the LDS position lpos (grouped by vertex, ascending (tet, corner)); each
    // of the block's free vertices sums its run into one partial; partial p
    // covers LDS positions [start, start + count) packed as start << 16 | count.
    std::vector<uint16_t> lpos;           // [nt][4], 0xFFFF for a pinned corner
    std::vector<int32_t> blk_part;        // nblocks+1: partial index ranges per block
    std::vector<int32_t> part_pack;       // per partial: start << 16 | count
    std::vector<int32_t> vpart_ptr, vpart;  // per free vertex: its partials (ascending)

    // FP64 free-free matrix in internal order (CSR) for refinement residuals;
    // the entry of each diagonal and each (element, corner a, corner b) pair
    // of free corners ([nt][4][4], -1 for a pinned corner)
    std::vector<int32_t> K_ptr, K_col;
    std::vector<double> K_val;
    std::vector<int32_t> K_diag, K_pair;

    // factor and solve programs
    std::vector<Supernode> sn;
    int64_t nnz_int = 0, nnz_coarse = 0;
    int32_t n_clevels = 0, max_sub_phases = 0, max_sub_n = 0;
    // interior: LDS chunk programs per subdomain
    std::vector<Chunk> chunks;
    std::vector<int32_t> sub_fwd_ch, sub_bwd_ch;   // D+1 ranges into chunks
    std::vector<float> ivals;                      // packed chunks (values and int words)
    std::vector<int32_t> bnd, bnd_off;             // per subdomain: interface rows it touches
    int32_t max_nb = 0, max_cint = 0, chunk_floats = 0;
    // interface: FP64 values and one launch per phase
    std::vector<double> dvals;
    std::vector<CTask> ctasks;
    std::vector<int32_t> cslots, cgidx;            // (unused: slots are contiguous per row), gather lists
    std::vector<CPhase> cfwd, cbwd;
    int32_t n_cgf = 0, n_cgd = 0;                  // global FP32 / FP64 contribution slots

    // refactorization with new stiffness (refactor_plan): the number of FP64
    // interior values, and for every word of ivals the interior value it
    // holds as FP32 (-1: a descriptor or index word)
    int64_t n_ivd = 0;
    std::vector<int32_t> ival_src;
    // interface supernodes factored on the device (PlanOptions::iface_on_device):
    // the update matrices of interior supernodes whose parent is an interface
    // supernode ([nsn], row-major upper m x m, empty otherwise) are kept for
    // it, and dvals holds the interface factor only once dvals_ready is set
    bool iface_on_device = false, dvals_ready = false;
    std::vector<std::vector<double>> iface_child_upd;

    double seconds = 0;
};

// Plan options.  thin_separators: separator vertices whose neighbours lie
// under one child only are eliminated inside that child's subtree.
// iface_on_device: the numeric factorization stops after the interior
// supernodes (the device factors the interface ones).
// merge_max_cols: the separators at odd depths join their parent's when the
// merged block has at most this many columns (0: no merging).  Tuning of the
// interface programs: a phase whose mean task length is at least lanes32_min
// (lanes64_min) runs 32 (64) lanes per task, else 16.
struct PlanOptions {
    bool thin_separators = true;
    bool iface_on_device = false;   // leave the interface numeric factorization to the device
    int64_t merge_max_cols = 3000;
    int64_t lanes32_min = 96, lanes64_min = 384;
};

// The inexact CMS solve of Sec. 7.2 (host data): per subdomain d, with n_d
// interior rows and nb_d adjacent interface rows (Plan::bnd), the interior
// eigenmodes Phi_d (modes columns of n_d, column-major at phi_off[d]), their
// inverse eigenvalues, the boundary modes Psi_d = -(K_d^ii)^{-1} K_d^ib
// (nb_d columns of n_d, column-major at psi_off[d]); for the Jacobi sweeps the
// inverse diagonal of K, the spectral radius rho of I - D^{-1} K and the
// Chebyshev weights omega_1..omega_sweeps.
struct CmsPlan {
    int32_t modes = 0, sweeps = 0;
    double rho = 0.0;
    std::vector<double> omega;
    std::vector<int64_t> phi_off, psi_off;
    std::vector<float> phi, psi, ilam;     // ilam: [D][modes] (0 past a subdomain's size)
    std::vector<double> lambda;            // [D][modes] FP64 eigenvalues (reports)
    std::vector<double> inv_diag;          // [n_free]
};
// Returns 0, or a negative VH_E* code with msg set.
int build_cms(const Plan& plan, int32_t modes, int32_t sweeps, CmsPlan& cms, std::string& msg);

// Build a plan; returns 0 or a negative VH_E* code with msg set.
int build_plan(const double* X, int32_t nv, const int32_t* tets, int32_t nt,
               const double* gamma_s, const double* gamma_v, const double* mass,
               const uint8_t* pinned, const double* gravity, double dt, int32_t pd_iters,
               int32_t n_subdomains, int32_t refine_steps, int32_t leaf_max,
               int32_t chunk_floats, const PlanOptions& opt, Plan& plan, std::string& msg);

// New per-element stiffness for a built plan of the same mesh (X, tets in
// user order): element weights, matrix values and the numeric factorization
// are redone; partition, orderings, supernodes and programs are kept, their
// values refreshed in place.  0 or a negative VH_E* code with msg set.
int refactor_plan(Plan& P, const double* X, const int32_t* tets, const double* gamma_s, const double* gamma_v,
                  std::string& msg);

// Rest-shape checks used at mesh creation: every tet has positive volume.
int check_mesh(const double* X, int32_t nv, const int32_t* tets, int32_t nt, std::string& msg);

}  // namespace vh
