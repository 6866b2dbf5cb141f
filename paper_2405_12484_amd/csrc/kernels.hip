// HIP kernels of the projective-dynamics step for CDNA4 (gfx950, wave64).
//
//   k_predict   Sec. 7: inertial target y = x* + dt v* + dt^2 g, x^(0) = y
//   k_local     Sec. 7.1 local step: per tet F, signed SVD, polar rotation R,
//               volume projection (Eq. vol_pre), residual stress and corner
//               forces, summed per vertex inside each workgroup (LDS, fixed order)
//   vertex_residual
//               Sec. 7.1 global step right-hand side, as the residual
//               r = b - K x^(k): per vertex the sum of its workgroup partials,
//               without atomics; in the PD iterations the first stage of
//               k_interior_fwd, as its own launch k_residual elsewhere
//   k_interior_fwd / k_coarse / k_interior_bwd
//               Sec. 7.2 decomposed solve K d = r: interior triangular
//               solves (one workgroup per subdomain, factor chunks and vectors
//               in LDS, FP32), interface solve (FP64, one launch per tree level
//               and task kind), interior back-substitution with the interface
//               values, x += d
//   k_refine    r -= K d in FP64 (optional refinement passes)
//   k_velocity  BDF1 velocity, non-finite check
#include "kernels.h"

namespace vh {

namespace {

constexpr int BLK = 256;

// Global views of generic pointers.  Pointers read from a descriptor table are
// generic, and an access through a generic pointer is a FLAT instruction,
// which counts against the LDS wait counter as well as the vector-memory one:
// in a kernel that also uses LDS, every wait for an LDS read would then wait
// for all global loads still in flight (a prefetch among them).
#define VH_GLOBAL __attribute__((address_space(1)))
template <class T>
__device__ __forceinline__ const VH_GLOBAL T* as_global(const T* p) {
    return (const VH_GLOBAL T*)p;
}
template <class T>
__device__ __forceinline__ VH_GLOBAL T* as_global(T* p) {
    return (VH_GLOBAL T*)p;
}
// Whole 16-byte records go through native vector types: HIP's float4 and int4
// are classes whose copy operations take generic references.
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef int32_t i32x4 __attribute__((ext_vector_type(4)));
__device__ __forceinline__ f32x4 load_global4(const float4* p) {
    return *reinterpret_cast<const VH_GLOBAL f32x4*>(as_global(p));
}
__device__ __forceinline__ void store_global4(float4* p, float x, float y, float z, float w) {
    *reinterpret_cast<VH_GLOBAL f32x4*>(as_global(p)) = f32x4{x, y, z, w};
}

// A launch covers one or more garments.  Its table L holds one int4 per block:
// {g: garment index into the DevMesh array, lb: block index within the
// garment, x0, x1: per-garment launch parameters}, so a block finds its
// garment with one load, and skips the work when the garment is not active in
// this launch.
struct Slot {
    int32_t g, lb, x0, x1;
};

__device__ __forceinline__ bool slot_of(const int32_t* __restrict__ L, const int32_t* __restrict__ active,
                                        Slot& s) {
    const int4 v = reinterpret_cast<const int4*>(L)[blockIdx.x];
    s.g = v.x;
    s.lb = v.y;
    s.x0 = v.z;
    s.x1 = v.w;
    return active[s.g] != 0;
}

// Hardware reciprocal / square root / reciprocal square root (about 1 ulp);
// every quantity they feed is FP32 and later compared at FP32 tolerance.
__device__ __forceinline__ float frcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ float fsqrt(float x) { return __builtin_amdgcn_sqrtf(x); }
__device__ __forceinline__ float frsq(float x) { return __builtin_amdgcn_rsqf(x); }

// ---------------------------------------------------------------------------
// 3x3 signed SVD in FP32: cyclic Jacobi eigen-decomposition of F^T F for W,
// then Givens QR of F W for U and the (signed) singular values; McAdams et al.
// (2011), "Computing the singular value decomposition of 3x3 matrices with
// minimal branching and elementary floating point operations", with exact
// Jacobi angles in place of their approximate quaternion ones.
// ---------------------------------------------------------------------------
// an off-diagonal below 2^-24 of its diagonal pair is negligible (no rotation);
// this also keeps denormals out of the hardware square root and reciprocal
__device__ __forceinline__ bool jacobi_negligible(float app, float aqq, float apq) {
    return !(fabsf(apq) > 5.96e-8f * (fabsf(app) + fabsf(aqq)) + 1e-30f);
}

// One Jacobi rotation zeroing apq.  With d = aqq - app, e = 2 apq and
// r = sqrt(d^2 + e^2), the smaller rotation has tan = t = sgn(d) e / (|d| + r),
// hence c = (|d| + r) w, s = sgn(d) e w and t = 2 r sgn(d) e w^2 with
// w = 1 / sqrt(2 r (|d| + r)): one square root and one reciprocal square root.
__device__ __forceinline__ void jacobi_pair(float& app, float& aqq, float& apq, float& arp,
                                            float& arq, float* W, int p, int q) {
    if (jacobi_negligible(app, aqq, apq)) return;
    const float d = aqq - app, ad = fabsf(d);
    const float e = (d < 0.0f) ? -2.0f * apq : 2.0f * apq;
    const float r = fsqrt(d * d + e * e);
    const float w = frsq(2.0f * r * (ad + r));
    const float c = (ad + r) * w;
    const float s = e * w;
    const float t = 2.0f * r * e * w * w;
    app -= t * apq;
    aqq += t * apq;
    apq = 0.0f;
    float rp = c * arp - s * arq;
    float rq = s * arp + c * arq;
    arp = rp;
    arq = rq;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        float wp = W[i * 3 + p], wq = W[i * 3 + q];
        W[i * 3 + p] = c * wp - s * wq;
        W[i * 3 + q] = s * wp + c * wq;
    }
}

__device__ __forceinline__ void swap_cols(float* W, int a, int b) {
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        float t = W[i * 3 + a];
        W[i * 3 + a] = W[i * 3 + b];
        W[i * 3 + b] = -t;   // keep det = +1
    }
}

// rows p, q of B (3x3 row-major): zero B[q][col] against B[p][col]; U <- U G^T
__device__ __forceinline__ void givens_rows(float* B, float* U, int p, int q, int col) {
    float a = B[p * 3 + col], b = B[q * 3 + col];
    float r2 = a * a + b * b;
    float c = 1.0f, s = 0.0f;
    if (r2 > 1e-37f) {
        float ir = frsq(r2);
        c = a * ir;
        s = b * ir;
    }
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        float bp = B[p * 3 + j], bq = B[q * 3 + j];
        B[p * 3 + j] = c * bp + s * bq;
        B[q * 3 + j] = -s * bp + c * bq;
    }
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        float up = U[i * 3 + p], uq = U[i * 3 + q];
        U[i * 3 + p] = c * up + s * uq;
        U[i * 3 + q] = -s * up + c * uq;
    }
}

__device__ __forceinline__ void svd3(const float* F, float* U, float* sig, float* W) {
    // A = F^T F
    float a00 = 0, a01 = 0, a02 = 0, a11 = 0, a12 = 0, a22 = 0;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        float f0 = F[k * 3 + 0], f1 = F[k * 3 + 1], f2 = F[k * 3 + 2];
        a00 += f0 * f0;
        a01 += f0 * f1;
        a02 += f0 * f2;
        a11 += f1 * f1;
        a12 += f1 * f2;
        a22 += f2 * f2;
    }
#pragma unroll
    for (int i = 0; i < 9; ++i) W[i] = (i % 4 == 0) ? 1.0f : 0.0f;
    // at most 4 sweeps; once every off-diagonal of every lane of the wave is
    // negligible, further sweeps would rotate nothing, so they are skipped
#pragma unroll
    for (int sweep = 0; sweep < 4; ++sweep) {
        if (sweep > 0 && __all(jacobi_negligible(a00, a11, a01) && jacobi_negligible(a00, a22, a02) &&
                               jacobi_negligible(a11, a22, a12)))
            break;
        jacobi_pair(a00, a11, a01, a02, a12, W, 0, 1);   // r = 2
        jacobi_pair(a00, a22, a02, a01, a12, W, 0, 2);   // r = 1: a10 = a01, a12 -> a21
        jacobi_pair(a11, a22, a12, a01, a02, W, 1, 2);   // r = 0: a01, a02
    }
    // sort eigenvalues descending (columns of W follow)
    float l0 = a00, l1 = a11, l2 = a22, t;
    if (l0 < l1) { t = l0; l0 = l1; l1 = t; swap_cols(W, 0, 1); }
    if (l0 < l2) { t = l0; l0 = l2; l2 = t; swap_cols(W, 0, 2); }
    if (l1 < l2) { t = l1; l1 = l2; l2 = t; swap_cols(W, 1, 2); }
    // B = F W, QR by Givens
    float B[9];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j)
            B[i * 3 + j] = F[i * 3 + 0] * W[0 * 3 + j] + F[i * 3 + 1] * W[1 * 3 + j] + F[i * 3 + 2] * W[2 * 3 + j];
#pragma unroll
    for (int i = 0; i < 9; ++i) U[i] = (i % 4 == 0) ? 1.0f : 0.0f;
    givens_rows(B, U, 0, 1, 0);
    givens_rows(B, U, 0, 2, 0);
    givens_rows(B, U, 1, 2, 1);
    sig[0] = B[0];
    sig[1] = B[4];
    sig[2] = B[8];
}

// s - sigma on the + branch s(mu) = (sigma + sqrt(sigma^2 + 4 mu)) / 2, written
// without cancellation; returns the root distance q = sqrt(sigma^2 + 4 mu).
__device__ __forceinline__ float plus_delta(float sg, float mu, float& q) {
    q = fsqrt(fmaxf(sg * sg + 4.0f * mu, 0.0f));
    if (sg >= 0.0f) return 2.0f * mu * frcp(q + sg);
    float s = 2.0f * mu * frcp(q - sg);
    return s - sg;
}

// Regime word of one projection: what happened beyond the plain + branch root.
// Bits 4..6 hold the mask of axes frozen by the clamp.
constexpr uint32_t kSl3Clamped = 1u, kSl3DetGe2 = 2u, kSl3Squash = 4u, kSl3NoPlus = 8u;
constexpr int kSl3FrozenShift = 4;
constexpr float kSl3Clamp = 0.01f;     // lower bound on a projected singular value (Sec. 7.1)

// ---- The rare regimes of Eq. vol_pre -----------------------------------------
// The Lagrange condition s_i (s_i - sigma_i) = mu has, per axis, the + root and,
// for mu < 0, the - root.  For a product target c over n free axes:
//   * the + branch (every axis on its + root) has at most one root of
//     prod s_i(mu) = c, since the product increases with mu;
//   * a mixed branch (axis k on its - root, mu in [-min sigma^2/4, 0)) can have
//     roots only when every sigma_i > 0 and prod sigma >= 2 c (there
//     s_k <= sigma_k / 2 and s_j <= sigma_j); two axes on the - root give
//     saddle points of the Lagrangian, never the nearest point.
// The nearest point is the candidate closest to sigma (ties: the + branch, then
// the lower axis, then the smaller |mu|).  The clamp of Sec. 7.1 sets a
// component below 0.01 to 0.01, freezes it, and solves the free axes again for
// the product 1 / 0.01^(frozen count).

// larger root of s^2 - sg s - mu = 0 without cancellation; q = sqrt(sg^2 + 4 mu)
__device__ __forceinline__ float plus_root(float sg, float mu, float& q) {
    q = sqrtf(fmaxf(sg * sg + 4.0f * mu, 0.0f));
    if (sg >= 0.0f) return 0.5f * (sg + q);
    return (q - sg > 0.0f) ? 2.0f * mu / (q - sg) : 0.0f;
}

// The free axes of a sub-problem are the set bits of `mask`.  s on the +
// branch (k < 0) or on the mixed branch with axis k on the - root at mu, and
// the product of its free components.
__device__ __forceinline__ float branch_point(const float* sg, uint32_t mask, int k, float mu, float* s) {
    float p = 1.0f;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        float q;
        const float sp = plus_root(sg[i], mu, q);
        s[i] = (i == k) ? -2.0f * mu / (sg[i] + q) : sp;
        if (mask >> i & 1u) p *= s[i];
    }
    return p;
}

// + branch root of prod s_i = c over the free axes (bisection down to
// adjacent floats); false when the branch has none
__device__ __forceinline__ bool plus_branch(const float* sg, uint32_t mask, float c, float* s) {
    float smin = INFINITY, det = 1.0f;
#pragma unroll
    for (int i = 0; i < 3; ++i)
        if (mask >> i & 1u) {
            smin = fminf(smin, sg[i]);
            det *= sg[i];
        }
    const bool grow = !(smin > 0.0f) || det <= c;          // root at mu >= 0
    float lo = grow ? 0.0f : -0.25f * smin * smin, hi = grow ? 1.0f : 0.0f;
    if (grow) {
#pragma unroll 1
        for (int k = 0; k < 260 && branch_point(sg, mask, -1, hi, s) <= c; ++k) hi = 2.0f * hi + 1.0f;
    } else if (branch_point(sg, mask, -1, lo, s) >= c) {
        return false;
    }
#pragma unroll 1
    for (int k = 0; k < 300; ++k) {
        const float mid = 0.5f * (lo + hi);
        if (!(mid > lo && mid < hi)) break;
        if (branch_point(sg, mask, -1, mid, s) > c) hi = mid;
        else lo = mid;
    }
    branch_point(sg, mask, -1, 0.5f * (lo + hi), s);
    return true;
}

// Roots of every mixed branch, found by a sign scan of prod s - c over mu at
// kSl3Scan geometric points from -1e-14 min sigma^2/4 down to -min sigma^2/4,
// then bisection of each sign change.  A root strictly nearer to sigma than
// d2 replaces (best, d2) on the free axes; returns whether one did.
constexpr int kSl3Scan = 1024;
__device__ __forceinline__ bool mixed_roots(const float* sg, uint32_t mask, float c, float* best, float& d2) {
    float smin = INFINITY, det = 1.0f;
#pragma unroll
    for (int i = 0; i < 3; ++i)
        if (mask >> i & 1u) {
            smin = fminf(smin, sg[i]);
            det *= sg[i];
        }
    if (!(smin > 0.0f) || det < 2.0f * c) return false;
    const float lo = -0.25f * smin * smin;
    const float ratio = 1.0320132f;        // 1e14^(1 / (kSl3Scan - 1))
    bool took = false;
    float s[3];
#pragma unroll 1
    for (int k = 0; k < 3; ++k) {
        if (!(mask >> k & 1u)) continue;
        float t = 1e-14f, mu_a = lo * t;
        float fa = branch_point(sg, mask, k, mu_a, s) - c;
#pragma unroll 1
        for (int j = 1; j < kSl3Scan; ++j) {
            t = (j == kSl3Scan - 1) ? 1.0f : t * ratio;
            const float mu_b = lo * t;
            const float fb = branch_point(sg, mask, k, mu_b, s) - c;
            if ((fa < 0.0f) != (fb < 0.0f)) {
                float a = mu_a, b = mu_b;
                const bool neg_a = fa < 0.0f;
#pragma unroll 1
                for (int it = 0; it < 300; ++it) {
                    const float m = 0.5f * (a + b);
                    if (!(m != a && m != b)) break;
                    if ((branch_point(sg, mask, k, m, s) - c < 0.0f) == neg_a) a = m;
                    else b = m;
                }
                branch_point(sg, mask, k, 0.5f * (a + b), s);
                float dd = 0.0f;
#pragma unroll
                for (int i = 0; i < 3; ++i)
                    if (mask >> i & 1u) dd += (s[i] - sg[i]) * (s[i] - sg[i]);
                if (dd < d2) {
                    d2 = dd;
#pragma unroll
                    for (int i = 0; i < 3; ++i)
                        if (mask >> i & 1u) best[i] = s[i];
                    took = true;
                }
            }
            mu_a = mu_b;
            fa = fb;
        }
    }
    return took;
}

// nearest point to sg on {product over the free axes of s = c, s > 0}, written
// to the free axes of s; adds kSl3NoPlus / kSl3Squash to *bits when the +
// branch has no root / a mixed root is nearer
__device__ __forceinline__ void nearest_on_product(const float* sg, uint32_t mask, float c, float* s,
                                                   uint32_t* bits) {
    if (__builtin_popcount(mask) == 1) {
#pragma unroll
        for (int i = 0; i < 3; ++i)
            if (mask >> i & 1u) s[i] = c;
        return;
    }
    float sp[3];
    const bool ok = plus_branch(sg, mask, c, sp);
    float d2 = INFINITY;
    if (ok) {
        d2 = 0.0f;
#pragma unroll
        for (int i = 0; i < 3; ++i)
            if (mask >> i & 1u) {
                s[i] = sp[i];
                d2 += (sp[i] - sg[i]) * (sp[i] - sg[i]);
            }
    } else {
        *bits |= kSl3NoPlus;
    }
    if (mixed_roots(sg, mask, c, s, d2)) *bits |= kSl3Squash;
}

// The projection outside the plain + branch: det F >= 2 (mixed stationary
// points may be nearer) or a component below the clamp.  FP32 like the rest of
// the local step, but by bracketing instead of a fixed count of Newton steps.
// Writes ds = s - sigma and returns the regime word.
__device__ __forceinline__ uint32_t proj_sl3_rare(const float* sg, float* ds) {
    float s[3] = {sg[0], sg[1], sg[2]};
    uint32_t bits = 0;
    if (sg[2] > 0.0f && sg[0] * sg[1] * sg[2] >= 2.0f) {
        bits |= kSl3DetGe2;
        nearest_on_product(sg, 7u, 1.0f, s, &bits);
    } else {
        plus_branch(sg, 7u, 1.0f, s);
    }
    uint32_t frozen = 0;
#pragma unroll 1
    for (int round = 0; round < 3; ++round) {
        uint32_t newly = 0;
#pragma unroll
        for (int i = 0; i < 3; ++i)
            if (!(frozen >> i & 1u) && s[i] < kSl3Clamp) newly |= 1u << i;
        if (!newly) break;
        frozen |= newly;
        const uint32_t free_axes = 7u & ~frozen;
        float c = 1.0f;
#pragma unroll
        for (int i = 0; i < 3; ++i)
            if (frozen >> i & 1u) {
                s[i] = kSl3Clamp;
                c *= 100.0f;               // 1 / kSl3Clamp
            }
        if (!free_axes) break;
        uint32_t sub_bits = 0;
        nearest_on_product(sg, free_axes, c, s, &sub_bits);
        bits |= sub_bits & kSl3Squash;
    }
    if (frozen) bits |= kSl3Clamped | (frozen << kSl3FrozenShift);
#pragma unroll
    for (int i = 0; i < 3; ++i) ds[i] = s[i] - sg[i];
    return bits;
}

// Nearest volume-preserving singular values (Eq. vol_pre): the Lagrange
// condition gives s_i (s_i - sigma_i) = mu for all i; Newton on
// h(mu) = ln(s1 s2 s3)(mu) from mu = 0, stop when |s1 s2 s3 - 1| is within
// 2 ulp of 1, at most kSl3Steps steps.  Near the root ln p is replaced by
// (p - 1)/p, which has the same root and slope.  Strains of a few percent take
// 3-4 steps; strongly compressed, nearly flat or inverted elements (sigma_3
// down to 1e-3, det F close to 2) take up to 10-12, and 16 leaves margin.
// Writes ds_i = s_i - sigma_i and returns false; returns true instead when
// det F >= 2 or a component lands below the clamp, where proj_sl3_rare decides.
constexpr int kSl3Steps = 16;
__device__ __forceinline__ bool proj_sl3_plus(const float* sg, float* ds) {
    float mu = (sg[2] > 0.0f) ? 0.0f : 0.25f;
    const float lo = (sg[2] > 0.0f) ? -0.25f * sg[2] * sg[2] : 0.0f;
    float q[3], s[3];
#pragma unroll 1
    for (int it = 0; it < kSl3Steps; ++it) {
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            ds[i] = plus_delta(sg[i], mu, q[i]);
            s[i] = sg[i] + ds[i];
        }
        float p = s[0] * s[1] * s[2];
        if (fabsf(p - 1.0f) < 2.4e-7f) break;
        // h' = sum_i 1 / (q_i s_i); with A_i = q_i s_i the Newton step h / h' is
        // h A1 A2 A3 / (A2 A3 + A1 A3 + A1 A2), and near the root h = (p - 1) / p
        const float A0 = q[0] * s[0], A1 = q[1] * s[1], A2 = q[2] * s[2];
        const float num = A0 * A1 * A2, den = A1 * A2 + A0 * A2 + A0 * A1;
        float step;
        if (fabsf(p - 1.0f) < 0.25f) step = (p - 1.0f) * num * frcp(p * den);
        else step = logf(p) * num * frcp(den);
        float mun = mu - step;
        if (!(mun > lo)) mun = 0.5f * (mu + lo);
        mu = mun;
        if (it == kSl3Steps - 1) {
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                ds[i] = plus_delta(sg[i], mu, q[i]);
                s[i] = sg[i] + ds[i];
            }
        }
    }
    return (sg[2] > 0.0f && sg[0] * sg[1] * sg[2] >= 2.0f) || s[0] < kSl3Clamp || s[1] < kSl3Clamp ||
           s[2] < kSl3Clamp;
}

// The projection of Eq. vol_pre with the clamp; returns the regime word.
__device__ __forceinline__ uint32_t proj_sl3(const float* sg, float* ds) {
    if (__builtin_expect(proj_sl3_plus(sg, ds), 0)) return proj_sl3_rare(sg, ds);
    return 0u;
}

// Per-element regime counters (64-bit): [0] clamped, [1] inverted (sigma_3 <= 0),
// [2] det F >= 2, [3] a mixed-branch point taken, [4] no + branch root.
__device__ __forceinline__ void count_regime(unsigned long long* regime, uint32_t bits, bool inverted) {
    if (bits & kSl3Clamped) atomicAdd(&regime[0], 1ull);
    if (inverted) atomicAdd(&regime[1], 1ull);
    if (bits & kSl3DetGe2) atomicAdd(&regime[2], 1ull);
    if (bits & kSl3Squash) atomicAdd(&regime[3], 1ull);
    if (bits & kSl3NoPlus) atomicAdd(&regime[4], 1ull);
}

// Local step, one thread per tet, 256 tets per workgroup.  Each tet reads
// one 64-byte record (vertex ids, Dm^{-1}, weights), gathers the four vertex
// displacements, and writes its four corner forces into LDS at positions that
// group them by vertex; the workgroup then sums each of its vertices' runs in
// a fixed order and stores one partial per (workgroup, vertex), coalesced.
constexpr int LBLK = 256;

// One tet's 64-byte record (vertex ids, Dm^{-1} rows, weights), its corner
// LDS positions, the gathered displacements, F = I + Du Dm^{-1}, and the signed
// SVD F = U diag(sg) W^T.
struct TetSvd {
    float G[9], ws, wv;
    uint2 lp;
    float U[9], W[9], sg[3];
};

__device__ __forceinline__ void tet_svd(const float4* __restrict__ trec, const uint2* __restrict__ lpos,
                                        const float4* __restrict__ u, int32_t e, TetSvd& t) {
    const float4 r0 = trec[4 * (size_t)e], r1 = trec[4 * (size_t)e + 1], r2 = trec[4 * (size_t)e + 2],
                 r3 = trec[4 * (size_t)e + 3];
    t.lp = lpos[e];
    const int32_t i0 = __float_as_int(r0.x), i1 = __float_as_int(r0.y), i2 = __float_as_int(r0.z),
                  i3 = __float_as_int(r0.w);
    const float4 u0 = u[i0], u1 = u[i1], u2 = u[i2], u3 = u[i3];
    const float G[9] = {r1.x, r1.y, r1.z, r1.w, r2.x, r2.y, r2.z, r2.w, r3.x};
#pragma unroll
    for (int k = 0; k < 9; ++k) t.G[k] = G[k];
    t.ws = r3.y;
    t.wv = r3.z;
    // displacement differences, columns k = corners 1..3
    const float Du[3][3] = {{u1.x - u0.x, u2.x - u0.x, u3.x - u0.x},
                            {u1.y - u0.y, u2.y - u0.y, u3.y - u0.y},
                            {u1.z - u0.z, u2.z - u0.z, u3.z - u0.z}};
    float F[9];
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int j = 0; j < 3; ++j)
            F[r * 3 + j] = (r == j ? 1.0f : 0.0f) + Du[r][0] * G[0 * 3 + j] + Du[r][1] * G[1 * 3 + j] +
                           Du[r][2] * G[2 * 3 + j];
    svd3(F, t.U, t.sg, t.W);
}

template <bool DBG>
__global__ __launch_bounds__(LBLK, 8) void k_local(const DevMesh* __restrict__ GM, const int32_t* __restrict__ L,
                                                const int32_t* __restrict__ active) {
    __shared__ float LF[3][4 * LBLK];
    Slot sl;
    if (!slot_of(L, active, sl)) return;
    const DevMesh& M = GM[sl.g];
    const int32_t nt = M.nt;
    const float4* __restrict__ trec = M.trec;
    const uint2* __restrict__ lpos = M.lpos;
    const float4* __restrict__ u = M.u;
    const int32_t* __restrict__ blk_part = M.blk_part;
    const int32_t* __restrict__ part_pack = M.part_pack;
    float4* __restrict__ part = M.part;
    float *dT = M.dbg_T, *dsig = M.dbg_sig, *ds_out = M.dbg_s;
    const int32_t e = sl.lb * LBLK + threadIdx.x;
    if (e < nt) {
        TetSvd t;
        tet_svd(trec, lpos, u, e, t);
        float dsv[3];
        uint32_t regime = 0;
        if (__builtin_expect(proj_sl3_plus(t.sg, dsv), 0)) {
            const float sg1[3] = {t.sg[0], t.sg[1], t.sg[2]};
            regime = proj_sl3_rare(sg1, dsv);
            // the record and the singular vectors are formed again (the same
            // values), so that only sigma stays live across the bracketing
            // and the kernel keeps the registers of the plain one
            __asm__ volatile("" ::: "memory");
            tet_svd(trec, lpos, u, e, t);
        }
        const float* G = t.G;
        const float *U = t.U, *W = t.W, *sg = t.sg;
        const float ws = t.ws, wv = t.wv;
        const uint2 lp = t.lp;
        // residual stress T = U diag(ws (1 - sigma) + wv (s - sigma)) W^T = P - (ws + wv) F
        const float d0 = ws * (1.0f - sg[0]) + wv * dsv[0];
        const float d1 = ws * (1.0f - sg[1]) + wv * dsv[1];
        const float d2 = ws * (1.0f - sg[2]) + wv * dsv[2];
        float T[9];
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = 0; j < 3; ++j)
                T[i * 3 + j] = U[i * 3 + 0] * d0 * W[j * 3 + 0] + U[i * 3 + 1] * d1 * W[j * 3 + 1] +
                               U[i * 3 + 2] * d2 * W[j * 3 + 2];
        // corner forces f_c = T gradN_c, gradN_c = row c-1 of Dm^{-1}, f_0 = -(f_1+f_2+f_3)
        const uint32_t pos[4] = {lp.x & 0xFFFFu, lp.x >> 16, lp.y & 0xFFFFu, lp.y >> 16};
        float s0 = 0, s1 = 0, s2 = 0;
#pragma unroll
        for (int c = 1; c < 4; ++c) {
            const float fx = T[0] * G[(c - 1) * 3 + 0] + T[1] * G[(c - 1) * 3 + 1] + T[2] * G[(c - 1) * 3 + 2];
            const float fy = T[3] * G[(c - 1) * 3 + 0] + T[4] * G[(c - 1) * 3 + 1] + T[5] * G[(c - 1) * 3 + 2];
            const float fz = T[6] * G[(c - 1) * 3 + 0] + T[7] * G[(c - 1) * 3 + 1] + T[8] * G[(c - 1) * 3 + 2];
            if (pos[c] != 0xFFFFu) {
                LF[0][pos[c]] = fx;
                LF[1][pos[c]] = fy;
                LF[2][pos[c]] = fz;
            }
            s0 += fx;
            s1 += fy;
            s2 += fz;
        }
        if (pos[0] != 0xFFFFu) {
            LF[0][pos[0]] = -s0;
            LF[1][pos[0]] = -s1;
            LF[2][pos[0]] = -s2;
        }
        const bool inv = sg[2] <= 0.0f;
        if (__builtin_expect(regime != 0u || inv, 0)) count_regime(M.regime, regime, inv);
        if (DBG) {
#pragma unroll
            for (int k = 0; k < 9; ++k) dT[(size_t)e * 9 + k] = T[k];
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                dsig[(size_t)e * 3 + k] = sg[k];
                ds_out[(size_t)e * 3 + k] = sg[k] + dsv[k];
            }
        }
    }
    __syncthreads();
    const int32_t p0 = blk_part[sl.lb], np = blk_part[sl.lb + 1] - p0;
    for (int32_t k = threadIdx.x; k < np; k += LBLK) {
        const int32_t pk = part_pack[p0 + k];
        const int32_t st = pk >> 16, cnt = pk & 0xFFFF;
        float fx = 0.0f, fy = 0.0f, fz = 0.0f;
        for (int32_t q = st; q < st + cnt; ++q) {
            fx += LF[0][q];
            fy += LF[1][q];
            fz += LF[2][q];
        }
        part[p0 + k] = make_float4(fx, fy, fz, 0.0f);
    }
}

// Cross-check of the scatter above (the alternative the partial sums replace):
// the tets of one colour share no free vertex, so each adds its four corner
// forces straight into the vertex sums.  The forces are formed from the stress
// the debug local step stored, with the expressions of k_local.
__global__ __launch_bounds__(BLK) void k_scatter_colour(const float4* __restrict__ trec, const float* __restrict__ T,
                                                        const int32_t* __restrict__ list, int32_t count,
                                                        int32_t n_free, float* __restrict__ b) {
    const int32_t j = blockIdx.x * BLK + threadIdx.x;
    if (j >= count) return;
    const int32_t e = list[j];
    const float4 r0 = trec[4 * (size_t)e], r1 = trec[4 * (size_t)e + 1], r2 = trec[4 * (size_t)e + 2],
                 r3 = trec[4 * (size_t)e + 3];
    const int32_t v[4] = {__float_as_int(r0.x), __float_as_int(r0.y), __float_as_int(r0.z), __float_as_int(r0.w)};
    const float G[9] = {r1.x, r1.y, r1.z, r1.w, r2.x, r2.y, r2.z, r2.w, r3.x};
    float t[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) t[k] = T[(size_t)e * 9 + k];
    float s0 = 0, s1 = 0, s2 = 0;
#pragma unroll
    for (int c = 1; c < 4; ++c) {
        const float fx = t[0] * G[(c - 1) * 3 + 0] + t[1] * G[(c - 1) * 3 + 1] + t[2] * G[(c - 1) * 3 + 2];
        const float fy = t[3] * G[(c - 1) * 3 + 0] + t[4] * G[(c - 1) * 3 + 1] + t[5] * G[(c - 1) * 3 + 2];
        const float fz = t[6] * G[(c - 1) * 3 + 0] + t[7] * G[(c - 1) * 3 + 1] + t[8] * G[(c - 1) * 3 + 2];
        if (v[c] < n_free) {
            b[3 * (size_t)v[c] + 0] += fx;
            b[3 * (size_t)v[c] + 1] += fy;
            b[3 * (size_t)v[c] + 2] += fz;
        }
        s0 += fx;
        s1 += fy;
        s2 += fz;
    }
    if (v[0] < n_free) {
        b[3 * (size_t)v[0] + 0] += -s0;
        b[3 * (size_t)v[0] + 1] += -s1;
        b[3 * (size_t)v[0] + 2] += -s2;
    }
}

__global__ __launch_bounds__(BLK) void k_predict(const DevMesh* __restrict__ GM, const int32_t* __restrict__ L,
                                                 const int32_t* __restrict__ active) {
    Slot sl;
    if (!slot_of(L, active, sl)) return;
    const DevMesh& M = GM[sl.g];
    const int32_t nv = M.nv, n_free = M.n_free;
    const double dt = M.dt;
    double* __restrict__ x = M.x;
    const double* __restrict__ v = M.v;
    double* __restrict__ xprev = M.xprev;
    double* __restrict__ y = M.y;
    const double* __restrict__ X = M.X;
    float4* __restrict__ u = M.u;
    const int32_t i = sl.lb * BLK + threadIdx.x;
    if (i >= nv) return;
    const double g[3] = {M.g[0], M.g[1], M.g[2]};
    float du[3];
    if (i < n_free) {
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            double xv = x[3 * i + c];
            double yv = xv + dt * v[3 * i + c] + dt * dt * g[c];
            xprev[3 * i + c] = xv;
            y[3 * i + c] = yv;
            x[3 * i + c] = yv;
            du[c] = (float)(yv - X[3 * i + c]);
        }
    } else {
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            double Xv = X[3 * i + c];
            xprev[3 * i + c] = Xv;
            y[3 * i + c] = Xv;
            x[3 * i + c] = Xv;
            du[c] = 0.0f;
        }
    }
    u[i] = make_float4(du[0], du[1], du[2], 0.0f);
}

// r_a = m_a (y_a - x_a) / dt^2 + the sum of the vertex's per-workgroup force
// partials (ascending workgroup order, so the result is deterministic).  The
// PD iterations compute it inside the interior forward solve (its prologue);
// this kernel serves the debug and timing entry points.
// (The pointers are plain or global-qualified views of the same arrays.)
template <class IP, class FP, class DP>
__device__ __forceinline__ void vertex_residual(IP vpart_ptr, IP vpart, FP part, DP mass, DP x, DP y, double inv_dt2,
                                                int32_t a, double& r0, double& r1, double& r2) {
    const int32_t j0 = vpart_ptr[a], j1 = vpart_ptr[a + 1];
    float fx = 0.0f, fy = 0.0f, fz = 0.0f;
    // up to four partials per round: their indices, then their values, are
    // loaded together (most vertices have one to three); absent ones add +0
    for (int32_t j = j0; j < j1; j += 4) {
        int32_t id[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) id[u] = (j + u < j1) ? vpart[j + u] : -1;
        f32x4 f[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) f[u] = (id[u] >= 0) ? part[id[u]] : f32x4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            fx += f[u].x;
            fy += f[u].y;
            fz += f[u].z;
        }
    }
    const double m = mass[a] * inv_dt2;
    r0 = m * (y[3 * a + 0] - x[3 * a + 0]) + (double)fx;
    r1 = m * (y[3 * a + 1] - x[3 * a + 1]) + (double)fy;
    r2 = m * (y[3 * a + 2] - x[3 * a + 2]) + (double)fz;
}

__global__ __launch_bounds__(BLK) void k_residual(const DevMesh* __restrict__ GM, const int32_t* __restrict__ L,
                                                  const int32_t* __restrict__ active) {
    Slot sl;
    if (!slot_of(L, active, sl)) return;
    const DevMesh& M = GM[sl.g];
    const int32_t a = sl.lb * BLK + threadIdx.x;
    if (a >= M.n_free) return;
    double r0, r1, r2;
    vertex_residual(M.vpart_ptr, M.vpart, reinterpret_cast<const f32x4*>(M.part), M.mass, M.x, M.y,
                    1.0 / (M.dt * M.dt), a, r0, r1, r2);
    double* __restrict__ r = M.r;
    r[3 * a + 0] = r0;
    r[3 * a + 1] = r1;
    r[3 * a + 2] = r2;
}

// Embedded points (Eq. m2y): p = N x over the four vertices of the point's tet,
// evaluated as x_0 + sum_{a=1..3} N_a (x_a - x_0) in FP64 with N_1..3 stored as
// FP32 (N_0 = 1 - N_1 - N_2 - N_3 is implied).  Records: two float4 per point,
// {v0, v1, v2, v3} (internal vertex ids, as int bits) and {N_1, N_2, N_3, 0}.
__global__ __launch_bounds__(BLK) void k_embed(const float4* __restrict__ rec, const double* __restrict__ x,
                                               int32_t n, double* __restrict__ out) {
    const int32_t i = blockIdx.x * BLK + threadIdx.x;
    if (i >= n) return;
    const float4 r0 = rec[2 * (size_t)i], r1 = rec[2 * (size_t)i + 1];
    const double* x0 = x + 3 * (size_t)__float_as_int(r0.x);
    const double* x1 = x + 3 * (size_t)__float_as_int(r0.y);
    const double* x2 = x + 3 * (size_t)__float_as_int(r0.z);
    const double* x3 = x + 3 * (size_t)__float_as_int(r0.w);
    const double n1 = r1.x, n2 = r1.y, n3 = r1.z;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const double b = x0[c];
        out[3 * (size_t)i + c] = b + n1 * (x1[c] - b) + n2 * (x2[c] - b) + n3 * (x3[c] - b);
    }
}

// ---------------------------------------------------------------------------
// Discrete adjoint of the PD iteration with respect to gamma_s (one garment).
// For x^(k+1) = L^{-1} b(x^(k)) and lambda = L^{-1} xbar^(k+1):
//   gbar_e  += V_e <G_e lambda, R_e(x^(k)) - F_e(x^(k+1))>   (b and L depend on gamma_s)
//   xbar^(k) = sum_e G_e^T dP_e,  dP_e = J_P(F_e(x^(k))) [G_e lambda]
// with P = w_s R + w_v V.  J_P is symmetric (R and V are projections), so the
// transposed product is this directional derivative.  In the singular bases
// (M = U^T dF W, a / b its symmetric / skew parts, s = Proj_SL3(sigma),
// q_i = sqrt(sigma_i^2 + 4 mu) = sigma_i + 2 (s_i - sigma_i)):
//   U^T dR W:  off-diagonal 2 b_ij / (sigma_i + sigma_j), diagonal 0
//   U^T dV W:  off-diagonal a_ij (1/2 + (sigma_i + sigma_j) / (2 (q_i + q_j)))
//                         + b_ij (s_i + s_j) / (sigma_i + sigma_j),
//              diagonal ds_i = (dmu + s_i M_ii) / q_i,
//              dmu = -(sum_i M_ii / q_i) / (sum_i 1 / (q_i s_i))
// (the divided difference (s_j - s_i) / (sigma_j - sigma_i) at the common mu is
// written without the difference, so equal singular values are harmless).
// ---------------------------------------------------------------------------
__device__ __forceinline__ void tet_F(const double* __restrict__ x, const double* __restrict__ X, const int32_t* id,
                                      const float* G, bool identity, float* F) {
    float u[4][3];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int c = 0; c < 3; ++c)
            u[a][c] = X ? (float)(x[3 * id[a] + c] - X[3 * id[a] + c]) : (float)x[3 * id[a] + c];
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int j = 0; j < 3; ++j)
            F[r * 3 + j] = (identity && r == j ? 1.0f : 0.0f) + (u[1][r] - u[0][r]) * G[0 * 3 + j] +
                           (u[2][r] - u[0][r]) * G[1 * 3 + j] + (u[3][r] - u[0][r]) * G[2 * 3 + j];
}

__global__ __launch_bounds__(LBLK) void k_adj_local(const DevMesh* __restrict__ GM, const double* __restrict__ xk,
                                                    const double* __restrict__ xk1,
                                                    const double* __restrict__ lam, double* __restrict__ gbar) {
    __shared__ float LF[3][4 * LBLK];
    const DevMesh& M = GM[0];
    const int32_t nt = M.nt;
    const int32_t e = blockIdx.x * LBLK + threadIdx.x;
    if (e < nt) {
        const float4* rec = M.trec + 4 * (size_t)e;
        const float4 r0 = rec[0], r1 = rec[1], r2 = rec[2], r3 = rec[3];
        const int32_t id[4] = {__float_as_int(r0.x), __float_as_int(r0.y), __float_as_int(r0.z),
                               __float_as_int(r0.w)};
        const float G[9] = {r1.x, r1.y, r1.z, r1.w, r2.x, r2.y, r2.z, r2.w, r3.x};
        const float ws = r3.y, wv = r3.z, Ve = r3.w;
        float F[9], F1[9], Gl[9];
        tet_F(xk, M.X, id, G, true, F);
        tet_F(xk1, M.X, id, G, true, F1);
        tet_F(lam, nullptr, id, G, false, Gl);
        float U[9], W[9], sg[3], dsv[3];
        svd3(F, U, sg, W);
        const uint32_t regime = proj_sl3(sg, dsv);
        const uint32_t frozen = regime >> kSl3FrozenShift;
        float s[3], q[3];
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            s[i] = sg[i] + dsv[i];
            q[i] = sg[i] + 2.0f * dsv[i];
        }
        // gamma_s term: V_e <G lambda, R - F(x^(k+1))>, R = U W^T
        float gs = 0.0f;
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = 0; j < 3; ++j) {
                const float Rij = U[i * 3 + 0] * W[j * 3 + 0] + U[i * 3 + 1] * W[j * 3 + 1] + U[i * 3 + 2] * W[j * 3 + 2];
                gs += Gl[i * 3 + j] * (Rij - F1[i * 3 + j]);
            }
        gbar[e] += (double)(Ve * gs);
        // M = U^T (G lambda) W
        float T1[9], Mm[9];
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = 0; j < 3; ++j)
                T1[i * 3 + j] = Gl[i * 3 + 0] * W[0 * 3 + j] + Gl[i * 3 + 1] * W[1 * 3 + j] + Gl[i * 3 + 2] * W[2 * 3 + j];
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = 0; j < 3; ++j)
                Mm[i * 3 + j] = U[0 * 3 + i] * T1[0 * 3 + j] + U[1 * 3 + i] * T1[1 * 3 + j] + U[2 * 3 + i] * T1[2 * 3 + j];
        // Q = U^T dP W = w_s U^T dR W + w_v U^T dV W
        float Q[9];
        {
            float sq = 0.0f, sis = 0.0f;
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                if (frozen >> i & 1u) continue;
                sq += Mm[i * 4] * frcp(q[i]);
                sis += frcp(q[i] * s[i]);
            }
            const float dmu = -sq * frcp(sis);
#pragma unroll
            for (int i = 0; i < 3; ++i)
                Q[i * 4] = (frozen >> i & 1u) ? 0.0f : wv * (dmu + s[i] * Mm[i * 4]) * frcp(q[i]);
        }
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = 0; j < 3; ++j) {
                if (i == j) continue;
                const float a = 0.5f * (Mm[i * 3 + j] + Mm[j * 3 + i]);
                const float b = 0.5f * (Mm[i * 3 + j] - Mm[j * 3 + i]);
                const float isum = frcp(sg[i] + sg[j]);
                const float dR = 2.0f * b * isum;
                // (s_i - s_j) / (sigma_i - sigma_j): at a common mu without the
                // difference; across a frozen axis (mu differs) as written
                float dd;
                if (!((frozen >> i | frozen >> j) & 1u)) dd = 0.5f + 0.5f * (sg[i] + sg[j]) * frcp(q[i] + q[j]);
                else dd = (sg[i] != sg[j]) ? (s[i] - s[j]) / (sg[i] - sg[j]) : 0.0f;
                const float dV = a * dd + b * (s[i] + s[j]) * isum;
                Q[i * 3 + j] = ws * dR + wv * dV;
            }
        // dP = U Q W^T
        float T2[9], dP[9];
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = 0; j < 3; ++j)
                T2[i * 3 + j] = U[i * 3 + 0] * Q[0 * 3 + j] + U[i * 3 + 1] * Q[1 * 3 + j] + U[i * 3 + 2] * Q[2 * 3 + j];
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = 0; j < 3; ++j)
                dP[i * 3 + j] = T2[i * 3 + 0] * W[j * 3 + 0] + T2[i * 3 + 1] * W[j * 3 + 1] + T2[i * 3 + 2] * W[j * 3 + 2];
        // corner forces of dP, grouped by vertex in LDS as in the local step
        const uint2 lp = M.lpos[e];
        const uint32_t pos[4] = {lp.x & 0xFFFFu, lp.x >> 16, lp.y & 0xFFFFu, lp.y >> 16};
        float s0 = 0, s1 = 0, s2 = 0;
#pragma unroll
        for (int c = 1; c < 4; ++c) {
            const float fx = dP[0] * G[(c - 1) * 3 + 0] + dP[1] * G[(c - 1) * 3 + 1] + dP[2] * G[(c - 1) * 3 + 2];
            const float fy = dP[3] * G[(c - 1) * 3 + 0] + dP[4] * G[(c - 1) * 3 + 1] + dP[5] * G[(c - 1) * 3 + 2];
            const float fz = dP[6] * G[(c - 1) * 3 + 0] + dP[7] * G[(c - 1) * 3 + 1] + dP[8] * G[(c - 1) * 3 + 2];
            if (pos[c] != 0xFFFFu) {
                LF[0][pos[c]] = fx;
                LF[1][pos[c]] = fy;
                LF[2][pos[c]] = fz;
            }
            s0 += fx;
            s1 += fy;
            s2 += fz;
        }
        if (pos[0] != 0xFFFFu) {
            LF[0][pos[0]] = -s0;
            LF[1][pos[0]] = -s1;
            LF[2][pos[0]] = -s2;
        }
        const bool inv = sg[2] <= 0.0f;
        if (__builtin_expect(regime != 0u || inv, 0)) count_regime(M.regime, regime, inv);
    }
    __syncthreads();
    const int32_t p0 = M.blk_part[blockIdx.x], np = M.blk_part[blockIdx.x + 1] - p0;
    for (int32_t k = threadIdx.x; k < np; k += LBLK) {
        const int32_t pk = M.part_pack[p0 + k];
        const int32_t st = pk >> 16, cnt = pk & 0xFFFF;
        float fx = 0.0f, fy = 0.0f, fz = 0.0f;
        for (int32_t q2 = st; q2 < st + cnt; ++q2) {
            fx += LF[0][q2];
            fy += LF[1][q2];
            fz += LF[2][q2];
        }
        M.part[p0 + k] = make_float4(fx, fy, fz, 0.0f);
    }
}

// xbar^(k)[a] = sum of the vertex's partials (fixed order); ybar[a] += m_a lambda_a / dt^2
__global__ __launch_bounds__(BLK) void k_adj_gather(const DevMesh* __restrict__ GM, const double* __restrict__ lam,
                                                    double* __restrict__ xbar, double* __restrict__ ybar) {
    const DevMesh& M = GM[0];
    const int32_t a = blockIdx.x * BLK + threadIdx.x;
    if (a >= M.n_free) return;
    float fx = 0.0f, fy = 0.0f, fz = 0.0f;
    for (int32_t j = M.vpart_ptr[a]; j < M.vpart_ptr[a + 1]; ++j) {
        const float4 f = M.part[M.vpart[j]];
        fx += f.x;
        fy += f.y;
        fz += f.z;
    }
    const double m = M.mass[a] / (M.dt * M.dt);
    xbar[3 * a + 0] = (double)fx;
    xbar[3 * a + 1] = (double)fy;
    xbar[3 * a + 2] = (double)fz;
    ybar[3 * a + 0] += m * lam[3 * a + 0];
    ybar[3 * a + 1] += m * lam[3 * a + 1];
    ybar[3 * a + 2] += m * lam[3 * a + 2];
}

// frame boundaries of the reverse sweep (free rows only):
//   begin: xk = xbar + vbar / dt, xn = -vbar / dt, ybar = 0
//   end:   ybar += xk (x^(0) = y), xbar = xn + ybar, vbar = dt ybar
__global__ __launch_bounds__(BLK) void k_adj_frame(int32_t n3, double dt, int32_t begin, double* __restrict__ xbar,
                                                   double* __restrict__ vbar, double* __restrict__ xk,
                                                   double* __restrict__ xn, double* __restrict__ ybar) {
    const int32_t i = blockIdx.x * BLK + threadIdx.x;
    if (i >= n3) return;
    if (begin) {
        xk[i] = xbar[i] + vbar[i] / dt;
        xn[i] = -vbar[i] / dt;
        ybar[i] = 0.0;
    } else {
        const double yb = ybar[i] + xk[i];
        xbar[i] = xn[i] + yb;
        vbar[i] = dt * yb;
    }
}

// ---------------------------------------------------------------------------
// Adjoint Gauss-Newton (Sec. 6.2, Eq. gn, Eq. agn) at an equilibrium x of one
// implicit Euler step, g(x, gamma) = M (x - y) / dt^2 + sum_e G_e^T (w_s (F - R)
// + w_v (F - V)) = 0:
//   B = dg/dgamma_s,  column e = V_e G_e^T (F_e - R_e)
//   A = dg/dx = K - sum_e G_e^T J_P(F_e) G_e   (K the step matrix of Sec. 7.1)
// B^T v and the J_P term of A v come from k_adj_local (with x^(k) = x^(k+1)
// = x its gamma_s term is V_e <G_e v, R_e - F_e> = -(B^T v)_e); B d and K v
// are the kernels below.
// ---------------------------------------------------------------------------

// per-workgroup partials of B d: the corner forces of d_e V_e (F_e - R_e)
__global__ __launch_bounds__(LBLK) void k_gn_bd(const DevMesh* __restrict__ GM, const double* __restrict__ x,
                                                const double* __restrict__ dgam) {
    __shared__ float LF[3][4 * LBLK];
    const DevMesh& M = GM[0];
    const int32_t nt = M.nt;
    const int32_t e = blockIdx.x * LBLK + threadIdx.x;
    if (e < nt) {
        const float4* rec = M.trec + 4 * (size_t)e;
        const float4 r0 = rec[0], r1 = rec[1], r2 = rec[2], r3 = rec[3];
        const int32_t id[4] = {__float_as_int(r0.x), __float_as_int(r0.y), __float_as_int(r0.z),
                               __float_as_int(r0.w)};
        const float G[9] = {r1.x, r1.y, r1.z, r1.w, r2.x, r2.y, r2.z, r2.w, r3.x};
        const float c = (float)(dgam[e] * (double)r3.w);       // d_e V_e
        float F[9], U[9], W[9], sg[3];
        tet_F(x, M.X, id, G, true, F);
        svd3(F, U, sg, W);
        // d_e V_e (F - R) = U diag(d_e V_e (sigma - 1)) W^T
        float Mm[9];
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = 0; j < 3; ++j)
                Mm[i * 3 + j] = c * (U[i * 3 + 0] * (sg[0] - 1.0f) * W[j * 3 + 0] +
                                     U[i * 3 + 1] * (sg[1] - 1.0f) * W[j * 3 + 1] +
                                     U[i * 3 + 2] * (sg[2] - 1.0f) * W[j * 3 + 2]);
        const uint2 lp = M.lpos[e];
        const uint32_t pos[4] = {lp.x & 0xFFFFu, lp.x >> 16, lp.y & 0xFFFFu, lp.y >> 16};
        float s0 = 0, s1 = 0, s2 = 0;
#pragma unroll
        for (int cc = 1; cc < 4; ++cc) {
            const float fx = Mm[0] * G[(cc - 1) * 3 + 0] + Mm[1] * G[(cc - 1) * 3 + 1] + Mm[2] * G[(cc - 1) * 3 + 2];
            const float fy = Mm[3] * G[(cc - 1) * 3 + 0] + Mm[4] * G[(cc - 1) * 3 + 1] + Mm[5] * G[(cc - 1) * 3 + 2];
            const float fz = Mm[6] * G[(cc - 1) * 3 + 0] + Mm[7] * G[(cc - 1) * 3 + 1] + Mm[8] * G[(cc - 1) * 3 + 2];
            if (pos[cc] != 0xFFFFu) {
                LF[0][pos[cc]] = fx;
                LF[1][pos[cc]] = fy;
                LF[2][pos[cc]] = fz;
            }
            s0 += fx;
            s1 += fy;
            s2 += fz;
        }
        if (pos[0] != 0xFFFFu) {
            LF[0][pos[0]] = -s0;
            LF[1][pos[0]] = -s1;
            LF[2][pos[0]] = -s2;
        }
    }
    __syncthreads();
    const int32_t p0 = M.blk_part[blockIdx.x], np = M.blk_part[blockIdx.x + 1] - p0;
    for (int32_t k = threadIdx.x; k < np; k += LBLK) {
        const int32_t pk = M.part_pack[p0 + k];
        const int32_t st = pk >> 16, cnt = pk & 0xFFFF;
        float fx = 0.0f, fy = 0.0f, fz = 0.0f;
        for (int32_t q2 = st; q2 < st + cnt; ++q2) {
            fx += LF[0][q2];
            fy += LF[1][q2];
            fz += LF[2][q2];
        }
        M.part[p0 + k] = make_float4(fx, fy, fz, 0.0f);
    }
}

// (K x)_i over the FP64 CSR matrix for the three components of x ([n][3]):
// four entries per round have their columns, values and gathered x in flight
// together; the products are added in entry order.
__device__ __forceinline__ void csr_row3(const int32_t* __restrict__ Kp, const int32_t* __restrict__ Kc,
                                         const double* __restrict__ Kv, const double* __restrict__ x, int32_t i,
                                         double& s0, double& s1, double& s2) {
    int32_t t = Kp[i];
    const int32_t t1 = Kp[i + 1];
    for (; t + 3 < t1; t += 4) {
        const int32_t c0 = Kc[t], c1 = Kc[t + 1], c2 = Kc[t + 2], c3 = Kc[t + 3];
        const double v0 = Kv[t], v1 = Kv[t + 1], v2 = Kv[t + 2], v3 = Kv[t + 3];
        const double* q0 = x + 3 * (size_t)c0;
        const double* q1 = x + 3 * (size_t)c1;
        const double* q2 = x + 3 * (size_t)c2;
        const double* q3 = x + 3 * (size_t)c3;
        const double a0 = q0[0], a1 = q0[1], a2 = q0[2], b0 = q1[0], b1 = q1[1], b2 = q1[2];
        const double e0 = q2[0], e1 = q2[1], e2 = q2[2], g0 = q3[0], g1 = q3[1], g2 = q3[2];
        s0 += v0 * a0;
        s1 += v0 * a1;
        s2 += v0 * a2;
        s0 += v1 * b0;
        s1 += v1 * b1;
        s2 += v1 * b2;
        s0 += v2 * e0;
        s1 += v2 * e1;
        s2 += v2 * e2;
        s0 += v3 * g0;
        s1 += v3 * g1;
        s2 += v3 * g2;
    }
    for (; t < t1; ++t) {
        const double v = Kv[t];
        const double* q = x + 3 * (size_t)Kc[t];
        s0 += v * q[0];
        s1 += v * q[1];
        s2 += v * q[2];
    }
}

// out = K v - geo on the free rows (FP64; K over the free-free block)
__global__ __launch_bounds__(BLK) void k_gn_av(const DevMesh* __restrict__ GM, const double* __restrict__ v,
                                               const double* __restrict__ geo, double* __restrict__ out) {
    const DevMesh& M = GM[0];
    const int32_t i = blockIdx.x * BLK + threadIdx.x;
    if (i >= M.n_free) return;
    double s0 = 0, s1 = 0, s2 = 0;
    csr_row3(M.K_ptr, M.K_col, M.K_val, v, i, s0, s1, s2);
    out[3 * i] = s0 - geo[3 * i];
    out[3 * i + 1] = s1 - geo[3 * i + 1];
    out[3 * i + 2] = s2 - geo[3 * i + 2];
}

// FP64 vector helpers of the Krylov loops: y += a x; y = x + b y; partial dot
// products (one per workgroup, summed in a fixed order on the host)
__global__ __launch_bounds__(BLK) void k_gn_axpy(int32_t n, double a, const double* __restrict__ x,
                                                 double* __restrict__ y) {
    const int32_t i = blockIdx.x * BLK + threadIdx.x;
    if (i < n) y[i] += a * x[i];
}

__global__ __launch_bounds__(BLK) void k_gn_xpby(int32_t n, const double* __restrict__ x, double b,
                                                 double* __restrict__ y) {
    const int32_t i = blockIdx.x * BLK + threadIdx.x;
    if (i < n) y[i] = x[i] + b * y[i];
}

__global__ __launch_bounds__(BLK) void k_gn_dot(int32_t n, const double* __restrict__ x,
                                                const double* __restrict__ y, double* __restrict__ part) {
    __shared__ double red[BLK];
    double acc = 0.0;
    for (int32_t i = blockIdx.x * BLK + threadIdx.x; i < n; i += gridDim.x * BLK) acc += x[i] * y[i];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int32_t w = BLK / 2; w > 0; w >>= 1) {
        if ((int32_t)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

// ---------------------------------------------------------------------------
// Decomposed solve
// ---------------------------------------------------------------------------

template <int WIDTH, class T>
__device__ __forceinline__ T group_sum(T v) {
#pragma unroll
    for (int off = WIDTH / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, WIDTH);
    return v;
}

struct SolveArgs {
    int32_t n_int, n_gamma, D, max_n, max_nb, max_cint, desc_table;
    const int32_t *sub_off, *sub_fwd_ch, *sub_bwd_ch, *bnd, *bnd_off;
    const Chunk* chunks;
    const float* ivals;          // packed interior chunks
    const CTask* ctasks;
    const int32_t *cslots, *cgidx;
    const double* dvals;
    double* r;
    // the residual computed by the forward solve's prologue (vertex_residual)
    const int32_t *vpart_ptr, *vpart;
    const float4* part;
    const double *mass, *y;
    double dt;
    float* zf;                   // [n_int][3] interior z
    float* cgf;                  // [n_cgf][3] contributions of interior supernodes to interface rows
    double* cgd;                 // [n_cgd][3] contributions of interface supernodes
    double *rg, *zg, *dg, *delta, *x;
    const double* X;
    float4* u;
};

__host__ __device__ __forceinline__ SolveArgs solve_args(const DevMesh& m) {
    SolveArgs a;
    a.n_int = m.n_int;
    a.n_gamma = m.n_gamma;
    a.D = m.D;
    a.max_n = m.max_sub_n;
    a.max_nb = m.max_nb;
    a.max_cint = m.max_cint;
    a.desc_table = m.desc_table;
    a.sub_off = m.sub_off;
    a.sub_fwd_ch = m.sub_fwd_ch;
    a.sub_bwd_ch = m.sub_bwd_ch;
    a.bnd = m.bnd;
    a.bnd_off = m.bnd_off;
    a.chunks = m.chunks;
    a.ivals = m.ivals;
    a.ctasks = m.ctasks;
    a.cslots = m.cslots;
    a.cgidx = m.cgidx;
    a.dvals = m.dvals;
    a.r = m.r;
    a.vpart_ptr = m.vpart_ptr;
    a.vpart = m.vpart;
    a.part = m.part;
    a.mass = m.mass;
    a.y = m.y;
    a.dt = m.dt;
    a.zf = m.zf;
    a.cgf = m.cgf;
    a.cgd = m.cgd;
    a.rg = m.rg;
    a.zg = m.zg;
    a.dg = m.dg;
    a.delta = m.delta;
    a.x = m.x;
    a.X = m.X;
    a.u = m.u;
    return a;
}

// Interior kernels: one 1024-thread workgroup (16 waves) per subdomain.
constexpr int BLKI = 1024;
constexpr int NV4I = 3;                       // float4 per thread per chunk
constexpr int32_t CHI = NV4I * 4 * BLKI;      // chunk capacity in 32-bit words (48 KB)

// Coalesced copy of one chunk (nv4 float4) into registers / LDS.  Three
// named registers rather than an array: the array ends up in scratch memory.
static_assert(NV4I == 3, "chunk staging holds three float4 per thread");
struct ChunkRegs {
    float a0, a1, a2, a3, b0, b1, b2, b3, c0, c1, c2, c3;
};
// Loads are unconditional (indices clamped into the chunk, nv4 >= 1) so the
// registers are always defined; only the stores are predicated.  They are
// non-temporal: a solve streams the interior programs (about 90 MB for the
// 390K-tet shell) once, and as ordinary loads they pushed the interface
// factor, which both sweeps of every solve read, and the local step's
// element records out of L2 and the MALL (interface solve 1.00 -> 0.85 ms
// per frame with these loads streamed; the same hint on the interface
// factor's loads made it slower).
__device__ __forceinline__ void chunk_load(const float4* __restrict__ src_, int32_t nv4, ChunkRegs& reg) {
    const int32_t j = threadIdx.x, last = nv4 - 1;
    const VH_GLOBAL f32x4* src = reinterpret_cast<const VH_GLOBAL f32x4*>(as_global(src_));
    f32x4 t = __builtin_nontemporal_load(src + min(j, last));
    reg.a0 = t.x; reg.a1 = t.y; reg.a2 = t.z; reg.a3 = t.w;
    t = __builtin_nontemporal_load(src + min(j + BLKI, last));
    reg.b0 = t.x; reg.b1 = t.y; reg.b2 = t.z; reg.b3 = t.w;
    t = __builtin_nontemporal_load(src + min(j + 2 * BLKI, last));
    reg.c0 = t.x; reg.c1 = t.y; reg.c2 = t.z; reg.c3 = t.w;
}
// The stores fill the whole buffer (NV4I * BLKI float4, words past the chunk
// get copies of its last float4): unpredicated, they leave the wait-count pass
// no path on which a load could still be pending when its registers are
// reused, so the loads of the next chunk can stay in flight across a phase.
__device__ __forceinline__ void chunk_store(float4* dst, const ChunkRegs& reg) {
    const int32_t j = threadIdx.x;
    dst[j] = make_float4(reg.a0, reg.a1, reg.a2, reg.a3);
    dst[j + BLKI] = make_float4(reg.b0, reg.b1, reg.b2, reg.b3);
    dst[j + 2 * BLKI] = make_float4(reg.c0, reg.c1, reg.c2, reg.c3);
}

// Descriptors of a subdomain's first tab <= CHD chunks are copied to LDS at
// kernel start, so the chunk pipeline does not wait on a global descriptor
// read for them; later chunks read theirs from global memory.
constexpr int32_t CHD = 64;

// kind, ntasks, v0, nv of chunk c, read from global memory
__device__ __forceinline__ Chunk chunk_desc_global(const Chunk* __restrict__ chunks, int32_t c) {
    const i32x4 v = *reinterpret_cast<const VH_GLOBAL i32x4*>(as_global(chunks + c));
    Chunk K{};
    K.kind = v.x;
    K.ntasks = v.y;
    K.v0 = v.z;
    K.nv = v.w;
    return K;
}

__device__ __forceinline__ Chunk chunk_desc(const Chunk* __restrict__ chunks, const int4* cd, int32_t tab,
                                            int32_t c0, int32_t c) {
    Chunk K;
    if (c - c0 < tab) {
        const int4 v = cd[c - c0];
        K.kind = v.x;
        K.ntasks = v.y;
        K.v0 = v.z;
        K.nv = v.w;
    } else {
        // a non-temporal read cannot be merged with the LDS read above into
        // one FLAT load of a selected address (a plain one was)
        const i32x4 v = __builtin_nontemporal_load(reinterpret_cast<const VH_GLOBAL i32x4*>(as_global(chunks + c)));
        K.kind = v.x;
        K.ntasks = v.y;
        K.v0 = v.z;
        K.nv = v.w;
    }
    return K;
}

// The start of a subdomain's chunk program, issued at kernel entry so that it
// overlaps the staging of the subdomain's vectors: the first chunk's load into
// registers, and the copy of the chunk descriptors into the LDS table.
struct ChunkStart {
    Chunk K0;
    ChunkRegs ra;
};
__device__ __forceinline__ void chunk_first(const Chunk* __restrict__ chunks, const float4* __restrict__ iv4,
                                            int32_t c0, int32_t c1, int4* cd, int32_t tab, ChunkStart& st) {
    if (c0 >= c1) return;
    st.K0 = chunk_desc_global(chunks, c0);
    chunk_load(iv4 + st.K0.v0 / 4, (st.K0.nv + 3) / 4, st.ra);
    for (int32_t c = c0 + (int32_t)threadIdx.x; c < min(c1, c0 + tab); c += BLKI) {
        const Chunk K = chunk_desc_global(chunks, c);
        cd[c - c0] = make_int4(K.kind, K.ntasks, K.v0, K.nv);
    }
}

// Runs compute(K, buf, spare) over the chunks c0..c1-1 of one subdomain.
// Chunk c is computed from LDS buffer (c - c0) & 1 while chunk c + 1 waits in
// registers for the other buffer (`spare`, free during compute) and the loads
// of chunk c + 2 are in flight, so every chunk's global read has two phases of
// compute to complete.  compute is called by every thread; ends with a barrier.
template <class F>
__device__ __forceinline__ void chunk_pipeline(const Chunk* __restrict__ chunks, const float4* __restrict__ iv4,
                                               int32_t c0, int32_t c1, float* sm, int4* cd, int32_t tab,
                                               ChunkStart& st, F&& compute) {
    // st: chunk_first's first chunk (registers) and descriptor table (LDS)
    if (c0 >= c1) {
        __syncthreads();   // the caller's LDS writes before the pipeline stay ordered before its reads after
        return;
    }
    ChunkRegs& ra = st.ra;   // next chunk for buffer 1
    ChunkRegs rb;            // next chunk for buffer 0
    const int32_t last = c1 - 1;
    Chunk K0 = st.K0;
    __syncthreads();
    float* buf0 = sm;
    float* buf1 = sm + CHI;
    // Loads and stores are unconditional: past the last chunk they repeat it
    // into the buffer that is no longer read.  Conditional ones left the
    // wait-count pass a path on which staged registers looked pending, and it
    // then waited for every load in flight at the top of each phase.
    chunk_store(reinterpret_cast<float4*>(buf0), ra);
    Chunk N1 = chunk_desc(chunks, cd, tab, c0, min(c0 + 1, last));
    chunk_load(iv4 + N1.v0 / 4, (N1.nv + 3) / 4, ra);
    Chunk K1 = N1;
    __syncthreads();
    // Pairs of chunks; an odd last one is computed after the loop (an exit
    // in mid-loop gave the pass a path from it back to the loop top).
    int32_t c = c0;
    for (; c + 1 < c1; c += 2) {
        // chunk c in buffer 0, chunk c + 1 in ra
        const Chunk N0 = chunk_desc(chunks, cd, tab, c0, min(c + 2, last));
        chunk_load(iv4 + N0.v0 / 4, (N0.nv + 3) / 4, rb);
        compute(K0, buf0, buf1);
        chunk_store(reinterpret_cast<float4*>(buf1), ra);
        K1 = N1;
        __syncthreads();
        // chunk c + 1 in buffer 1, chunk c + 2 in rb
        N1 = chunk_desc(chunks, cd, tab, c0, min(c + 3, last));
        chunk_load(iv4 + N1.v0 / 4, (N1.nv + 3) / 4, ra);
        compute(K1, buf1, buf0);
        chunk_store(reinterpret_cast<float4*>(buf0), rb);
        K0 = N0;
        __syncthreads();
    }
    if (c < c1) {
        // the last chunk, in buffer 0
        compute(K0, buf0, buf1);
        __syncthreads();
    }
}

// Interior forward solve.  Per supernode level: PULLSUM (thread per row)
// r'_row -= sum of its LDS contribution slots; GEMV (lane per row of
// [Ti; B Ti], 64 rows per wave item) accumulating column by column of the
// column-major block against broadcast r' values: z to LDS, contributions to
// interior rows to LDS slots, to interface rows to global FP32 slots.  The next
// chunk is read into registers while the current one is computed.
__global__ __launch_bounds__(BLKI) void k_interior_fwd(const DevMesh* __restrict__ GM,
                                                        const int32_t* __restrict__ L,
                                                        const int32_t* __restrict__ active, int32_t resid) {
    Slot sl;
    if (!slot_of(L, active, sl)) return;
    const SolveArgs a = solve_args(GM[sl.g]);
    extern __shared__ float4 sm4[];
    float* sm = reinterpret_cast<float*>(sm4);
    int4* cd = reinterpret_cast<int4*>(sm + 2 * CHI);   // 16-byte aligned: CHI is a multiple of 4
    float* R = sm + 2 * CHI + 4 * CHD;
    float* Z = R + 3 * a.max_n;
    float* C = Z + 3 * a.max_n;
    const int32_t d = sl.lb;
    const int32_t base = as_global(a.sub_off)[d];
    const int32_t n_loc = as_global(a.sub_off)[d + 1] - base;
    const int tid = threadIdx.x;
    const int32_t c0 = as_global(a.sub_fwd_ch)[d], c1 = as_global(a.sub_fwd_ch)[d + 1];
    const int32_t tab = min(max(a.desc_table, 1), CHD);
    const float4* iv4 = reinterpret_cast<const float4*>(a.ivals);
    // the residual is staged before the chunk program starts: vector loads
    // complete in issue order, so chunk loads issued first would hold it up
    if (resid) {
        // r = b - L x of the PD iteration, computed here rather than by a
        // launch of its own: this subdomain's interior rows, and a slice of
        // the interface rows (the interface solve reads them from r)
        const int32_t q = (a.n_gamma + a.D - 1) / a.D;
        const int32_t g0 = a.n_int + min(d * q, a.n_gamma);
        const int32_t g1 = a.n_int + min((d + 1) * q, a.n_gamma);
        const double inv_dt2 = 1.0 / (a.dt * a.dt);
        for (int32_t i = tid; i < n_loc + (g1 - g0); i += BLKI) {
            const int32_t v = (i < n_loc) ? base + i : g0 + (i - n_loc);
            double r0, r1, r2;
            vertex_residual(as_global(a.vpart_ptr), as_global(a.vpart), as_global(reinterpret_cast<const f32x4*>(a.part)),
                            as_global(a.mass), as_global((const double*)a.x), as_global(a.y), inv_dt2, v, r0, r1, r2);
            VH_GLOBAL double* rp = as_global(a.r) + 3 * (size_t)v;
            rp[0] = r0;
            rp[1] = r1;
            rp[2] = r2;
            if (i < n_loc) {
                R[3 * i + 0] = (float)r0;
                R[3 * i + 1] = (float)r1;
                R[3 * i + 2] = (float)r2;
            }
        }
    } else {
        for (int32_t i = tid; i < 3 * n_loc; i += BLKI) R[i] = (float)as_global(a.r)[3 * base + i];
    }
    ChunkStart st;
    chunk_first(a.chunks, iv4, c0, c1, cd, tab, st);
    const int wave = tid / 64, lane = tid % 64;
    constexpr int NW = BLKI / 64;
    chunk_pipeline(a.chunks, iv4, c0, c1, sm, cd, tab, st, [&](const Chunk& K, const float* cur, float*) {
        const int32_t* desc = reinterpret_cast<const int32_t*>(cur);
        if (K.kind == PULLSUM) {
            const int32_t* idat = desc + 4 * K.ntasks;
            for (int32_t t = tid; t < K.ntasks; t += BLKI) {
                const int32_t* q = desc + 4 * t;
                const int32_t* sl = idat + q[1];
                const int32_t cnt = q[2];
                float s0 = 0.0f, s1 = 0.0f, s2 = 0.0f;
                // unrolled so that several slot indices are in flight at once
                // (the sum stays in slot order)
#pragma unroll 4
                for (int32_t k = 0; k < cnt; ++k) {
                    const float* cp = C + 3 * sl[k];
                    s0 += cp[0];
                    s1 += cp[1];
                    s2 += cp[2];
                }
                float* rp = R + 3 * q[0];
                rp[0] -= s0;
                rp[1] -= s1;
                rp[2] -= s2;
            }
        } else {
            const float* dat = cur + 8 * K.ntasks;
            for (int32_t t = wave; t < K.ntasks; t += NW) {
                const int32_t* q = desc + 8 * t;
                const int32_t col0 = q[0], n = q[1], m = q[2], mi = q[3];
                const int32_t i = q[7] + lane;
                if (i >= n + m) continue;
                const float* w = dat + q[6] + i;        // column k element of row i: w[co(k) - k]
                const float* x = R + 3 * col0;
                const int32_t kmax = min(i + 1, n), stride0 = n + m;
                float s0 = 0.0f, s1 = 0.0f, s2 = 0.0f;
                int32_t co = 0;
#pragma unroll 4
                for (int32_t k = 0; k < kmax; ++k) {
                    const float v = w[co - k];
                    s0 += v * x[3 * k];
                    s1 += v * x[3 * k + 1];
                    s2 += v * x[3 * k + 2];
                    co += stride0 - k;
                }
                if (i < n + mi) {
                    float* op = (i < n) ? Z + 3 * (col0 + i) : C + 3 * (q[4] + i - n);
                    op[0] = s0;
                    op[1] = s1;
                    op[2] = s2;
                } else {
                    const int32_t slot = reinterpret_cast<const int32_t*>(dat)[q[5] + i - n - mi];
                    VH_GLOBAL float* op = as_global(a.cgf) + 3 * (size_t)slot;
                    op[0] = s0;
                    op[1] = s1;
                    op[2] = s2;
                }
            }
        }
    });
    for (int32_t i = tid; i < 3 * n_loc; i += BLKI) as_global(a.zf)[3 * base + i] = Z[i];
}

// Interface phases, one group of G lanes per task (FP64).
//   PULLSUM: rg[row] = r[row] - sum of its FP32 slots - sum of its FP64 slots
//   GEMV:    zg[idx], cgd[idx] or (a root, rows of Ti^T Ti) dg[idx] = row . rg
//   BGEMV:   dg[out] = Ti column . zg + (-W_B) column . dg[gather]
template <int G>
__global__ __launch_bounds__(BLK, 8) void k_coarse(const DevMesh* __restrict__ GM, const int32_t* __restrict__ L,
                                                const int32_t* __restrict__ active, int32_t kind) {
    Slot sl;
    if (!slot_of(L, active, sl)) return;
    const SolveArgs a = solve_args(GM[sl.g]);
    const int32_t task0 = sl.x0, ntasks = sl.x1;
    const int grp = threadIdx.x / G, lane = threadIdx.x % G;
    const int32_t t = sl.lb * (BLK / G) + grp;
    if (t >= ntasks) return;
    CTask T;
    {
        const VH_GLOBAL i32x4* tp = reinterpret_cast<const VH_GLOBAL i32x4*>(as_global(a.ctasks + task0 + t));
        const i32x4 lo = tp[0], hi = tp[1];
        T.a[0] = lo.x; T.a[1] = lo.y; T.a[2] = lo.z; T.a[3] = lo.w;
        T.a[4] = hi.x; T.a[5] = hi.y; T.a[6] = hi.z; T.a[7] = hi.w;
    }
    double s0 = 0.0, s1 = 0.0, s2 = 0.0;
    if (kind == PULLSUM) {
        // the row's slots are two contiguous runs (FP32 from the interiors,
        // FP64 from interface supernodes)
        for (int32_t k = lane; k < T.a[2]; k += G) {
            const VH_GLOBAL float* cp = as_global(a.cgf) + 3 * ((size_t)T.a[1] + k);
            s0 += (double)cp[0];
            s1 += (double)cp[1];
            s2 += (double)cp[2];
        }
        for (int32_t k = lane; k < T.a[4]; k += G) {
            const VH_GLOBAL double* cp = as_global(a.cgd) + 3 * ((size_t)T.a[3] + k);
            s0 += cp[0];
            s1 += cp[1];
            s2 += cp[2];
        }
    } else if (kind == GEMV) {
        const VH_GLOBAL double* vp = as_global(a.dvals) + T.a[2];
        const VH_GLOBAL double* xb = as_global(a.rg) + 3 * T.a[4];
        const int32_t len = T.a[3];
        int32_t k = lane;
        for (; k + 3 * G < len; k += 4 * G) {
            const double v0 = vp[k], v1 = vp[k + G], v2 = vp[k + 2 * G], v3 = vp[k + 3 * G];
            const VH_GLOBAL double* x0 = xb + 3 * k;
            const VH_GLOBAL double* x1 = x0 + 3 * G;
            const VH_GLOBAL double* x2 = x1 + 3 * G;
            const VH_GLOBAL double* x3 = x2 + 3 * G;
            s0 += v0 * x0[0] + v1 * x1[0] + v2 * x2[0] + v3 * x3[0];
            s1 += v0 * x0[1] + v1 * x1[1] + v2 * x2[1] + v3 * x3[1];
            s2 += v0 * x0[2] + v1 * x1[2] + v2 * x2[2] + v3 * x3[2];
        }
        for (; k < len; k += G) {
            const double v = vp[k];
            const VH_GLOBAL double* xp = xb + 3 * k;
            s0 += v * xp[0];
            s1 += v * xp[1];
            s2 += v * xp[2];
        }
    } else {
        // four independent elements per lane and round keep enough loads in
        // flight; the per-lane summation order is fixed by the lane index
        const VH_GLOBAL double* vp = as_global(a.dvals) + T.a[1];
        const int32_t len1 = T.a[2], len2 = T.a[4];
        const VH_GLOBAL double* zb = as_global(a.zg) + 3 * T.a[3];
        int32_t k = lane;
        for (; k + 3 * G < len1; k += 4 * G) {
            const double v0 = vp[k], v1 = vp[k + G], v2 = vp[k + 2 * G], v3 = vp[k + 3 * G];
            const VH_GLOBAL double* x0 = zb + 3 * k;
            const VH_GLOBAL double* x1 = x0 + 3 * G;
            const VH_GLOBAL double* x2 = x1 + 3 * G;
            const VH_GLOBAL double* x3 = x2 + 3 * G;
            s0 += v0 * x0[0] + v1 * x1[0] + v2 * x2[0] + v3 * x3[0];
            s1 += v0 * x0[1] + v1 * x1[1] + v2 * x2[1] + v3 * x3[1];
            s2 += v0 * x0[2] + v1 * x1[2] + v2 * x2[2] + v3 * x3[2];
        }
        for (; k < len1; k += G) {
            const double v = vp[k];
            const VH_GLOBAL double* xp = zb + 3 * k;
            s0 += v * xp[0];
            s1 += v * xp[1];
            s2 += v * xp[2];
        }
        const VH_GLOBAL double* v2p = vp + len1;
        const VH_GLOBAL int32_t* gi = as_global(a.cgidx) + T.a[5];
        const VH_GLOBAL double* dgv = as_global(a.dg);
        k = lane;
        for (; k + 3 * G < len2; k += 4 * G) {
            const int32_t g0 = gi[k], g1 = gi[k + G], g2 = gi[k + 2 * G], g3 = gi[k + 3 * G];
            const double v0 = v2p[k], v1 = v2p[k + G], v2 = v2p[k + 2 * G], v3 = v2p[k + 3 * G];
            const VH_GLOBAL double* x0 = dgv + 3 * g0;
            const VH_GLOBAL double* x1 = dgv + 3 * g1;
            const VH_GLOBAL double* x2 = dgv + 3 * g2;
            const VH_GLOBAL double* x3 = dgv + 3 * g3;
            s0 += v0 * x0[0] + v1 * x1[0] + v2 * x2[0] + v3 * x3[0];
            s1 += v0 * x0[1] + v1 * x1[1] + v2 * x2[1] + v3 * x3[1];
            s2 += v0 * x0[2] + v1 * x1[2] + v2 * x2[2] + v3 * x3[2];
        }
        for (; k < len2; k += G) {
            const double v = v2p[k];
            const VH_GLOBAL double* xp = dgv + 3 * gi[k];
            s0 += v * xp[0];
            s1 += v * xp[1];
            s2 += v * xp[2];
        }
    }
    s0 = group_sum<G>(s0);
    s1 = group_sum<G>(s1);
    s2 = group_sum<G>(s2);
    if (lane == 0) {
        VH_GLOBAL double* op;
        if (kind == PULLSUM) {
            const VH_GLOBAL double* rp = as_global(a.r) + 3 * ((size_t)a.n_int + T.a[0]);
            op = as_global(a.rg) + 3 * T.a[0];
            op[0] = rp[0] - s0;
            op[1] = rp[1] - s1;
            op[2] = rp[2] - s2;
            return;
        }
        if (kind == GEMV) op = (T.a[0] == 0) ? as_global(a.zg) + 3 * T.a[1]
                               : (T.a[0] == 1) ? as_global(a.cgd) + 3 * (size_t)T.a[1] : as_global(a.dg) + 3 * T.a[1];
        else op = as_global(a.dg) + 3 * T.a[0];
        op[0] = s0;
        op[1] = s1;
        op[2] = s2;
    }
}

// Interior backward solve and update.  Per supernode level, top down: BGEMV
// (lanes per column k of the row-major block [Ti; B Ti], the rows split among
// them and combined by a fixed butterfly):
// d_k = sum_{i>=k} Ti[i][k] z_i - sum_p (B Ti)[p][k] d[rows_p], with the
// subdomain's boundary values of the interface solution staged in LDS after
// its interior rows, so every gather hits LDS.
__global__ __launch_bounds__(BLKI) void k_interior_bwd(const DevMesh* __restrict__ GM,
                                                        const int32_t* __restrict__ L,
                                                        const int32_t* __restrict__ active, int32_t apply,
                                                        int32_t keep_delta) {
    Slot sl;
    if (!slot_of(L, active, sl)) return;
    const SolveArgs a = solve_args(GM[sl.g]);
    extern __shared__ float4 sm4[];
    float* sm = reinterpret_cast<float*>(sm4);
    int4* cd = reinterpret_cast<int4*>(sm + 2 * CHI);   // 16-byte aligned: CHI is a multiple of 4
    float* Z = sm + 2 * CHI + 4 * CHD;
    float* DL = Z + 3 * a.max_n;
    const int32_t d = sl.lb;
    const int32_t base = as_global(a.sub_off)[d];
    const int32_t n_loc = as_global(a.sub_off)[d + 1] - base;
    const int32_t b0 = as_global(a.bnd_off)[d], nb = as_global(a.bnd_off)[d + 1] - b0;
    const int tid = threadIdx.x;
    const int32_t c0 = as_global(a.sub_bwd_ch)[d], c1 = as_global(a.sub_bwd_ch)[d + 1];
    const int32_t tab = min(max(a.desc_table, 1), CHD);
    const float4* iv4 = reinterpret_cast<const float4*>(a.ivals);
    ChunkStart st;
    chunk_first(a.chunks, iv4, c0, c1, cd, tab, st);
    for (int32_t i = tid; i < 3 * n_loc; i += BLKI) Z[i] = as_global(a.zf)[3 * base + i];
    for (int32_t i = tid; i < 3 * nb; i += BLKI) {
        const int32_t k = i / 3, c = i - 3 * k;
        DL[3 * n_loc + i] = (float)as_global(a.dg)[3 * (as_global(a.bnd)[b0 + k] - a.n_int) + c];
    }
    // this thread's first interior row: x and X fetched now for the update at the end
    double px[3] = {0.0, 0.0, 0.0}, pX[3] = {0.0, 0.0, 0.0};
    if (apply && tid < n_loc) {
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            px[c] = as_global(a.x)[3 * (size_t)(base + tid) + c];
            pX[c] = as_global(a.X)[3 * (size_t)(base + tid) + c];
        }
    }
    // a slice of the interface rows (their values are final): updated first,
    // while the first chunks load
    {
        const int32_t chunk = (a.n_gamma + a.D - 1) / a.D;
        const int32_t g0 = d * chunk, g1 = min(a.n_gamma, g0 + chunk);
        for (int32_t i = g0 + tid; i < g1; i += BLKI) {
            const int32_t gi = a.n_int + i;
            // all loads before the first store, which they could otherwise not pass
            double dv[3], xo[3] = {0.0, 0.0, 0.0}, Xo[3] = {0.0, 0.0, 0.0};
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                dv[c] = as_global(a.dg)[3 * i + c];
                if (apply) {
                    xo[c] = as_global(a.x)[3 * gi + c];
                    Xo[c] = as_global(a.X)[3 * gi + c];
                }
            }
            float du[3];
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                if (keep_delta) as_global(a.delta)[3 * gi + c] = dv[c];
                if (apply) {
                    const double xn = xo[c] + dv[c];
                    as_global(a.x)[3 * gi + c] = xn;
                    du[c] = (float)(xn - Xo[c]);
                }
            }
            if (apply) store_global4(a.u + gi, du[0], du[1], du[2], 0.0f);
        }
    }
    const int wave = tid / 64, lane = tid % 64;
    constexpr int NW = BLKI / 64;
    chunk_pipeline(a.chunks, iv4, c0, c1, sm, cd, tab, st, [&](const Chunk& K, const float* cur, float* spare) {
        const int32_t* desc = reinterpret_cast<const int32_t*>(cur);
        const float* dat = cur + 8 * K.ntasks;
        const int32_t* idat = reinterpret_cast<const int32_t*>(dat);
        // a phase with fewer tasks than waves gives each task wpt waves, each
        // taking every wpt-th group of rows; their column sums meet in `spare`
        int32_t wpt = 1;
        while (2 * wpt * K.ntasks <= NW) wpt *= 2;
        const int32_t sub = wave % wpt;
        for (int32_t t = wave / wpt; t < K.ntasks; t += NW / wpt) {
            const int32_t* q = desc + 8 * t;
            const int32_t col0 = q[0], n = q[1], m = q[2];
            // lanes per column: the wave's 64 lanes are split into `lpc` groups of
            // `ncp` columns (ncp >= n, a power of two); group j of sub-wave `sub`
            // takes rows j + lpc sub, j + lpc (sub + wpt), ...
            const int32_t ncp = (n <= 8) ? 8 : (n <= 16) ? 16 : (n <= 32) ? 32 : 64;
            const int32_t lpc = 64 / ncp, stride = lpc * wpt;
            const int32_t kl = lane & (ncp - 1), j = lane / ncp;
            const int32_t k = q[5] + kl;
            const bool act = k < n;
            const float* w = dat + q[3] + k;
            float s0 = 0.0f, s1 = 0.0f, s2 = 0.0f;
            if (act) {
                for (int32_t i = k + j + lpc * sub; i < n; i += stride) {
                    const float v = w[i * (i + 1) / 2];
                    const float* xp = Z + 3 * (col0 + i);
                    s0 += v * xp[0];
                    s1 += v * xp[1];
                    s2 += v * xp[2];
                }
                const float* wb = w + n * (n + 1) / 2;
                const int32_t* g = idat + q[4];
#pragma unroll 4
                for (int32_t p = j + lpc * sub; p < m; p += stride) {
                    const float v = wb[p * n];
                    const float* xp = DL + 3 * g[p];
                    s0 -= v * xp[0];
                    s1 -= v * xp[1];
                    s2 -= v * xp[2];
                }
            }
            for (int32_t off = ncp; off < 64; off <<= 1) {
                s0 += __shfl_xor(s0, off, 64);
                s1 += __shfl_xor(s1, off, 64);
                s2 += __shfl_xor(s2, off, 64);
            }
            if (act && j == 0) {
                float* op = (wpt == 1) ? DL + 3 * (col0 + k) : spare + 3 * (wave * 64 + kl);
                op[0] = s0;
                op[1] = s1;
                op[2] = s2;
            }
        }
        if (wpt > 1) {
            // every task had one round: sum its sub-waves' partials in order
            __syncthreads();
            const int32_t t = wave / wpt;
            if (sub == 0 && t < K.ntasks) {
                const int32_t* q = desc + 8 * t;
                const int32_t n = q[1];
                const int32_t ncp = (n <= 8) ? 8 : (n <= 16) ? 16 : (n <= 32) ? 32 : 64;
                const int32_t kl = lane & (ncp - 1), k = q[5] + kl;
                if (lane < ncp && k < n) {
                    float s0 = 0.0f, s1 = 0.0f, s2 = 0.0f;
                    for (int32_t u = 0; u < wpt; ++u) {
                        const float* pp = spare + 3 * ((wave + u) * 64 + kl);
                        s0 += pp[0];
                        s1 += pp[1];
                        s2 += pp[2];
                    }
                    float* op = DL + 3 * (q[0] + k);
                    op[0] = s0;
                    op[1] = s1;
                    op[2] = s2;
                }
            }
            __syncthreads();   // `spare` receives the next chunk after this phase
        }
    });
    // interior rows of this subdomain
    for (int32_t i = tid; i < n_loc; i += BLKI) {
        const int32_t gi = base + i;
        const bool first = (i == tid);
        float du[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const double dv = (double)DL[3 * i + c];
            if (keep_delta) as_global(a.delta)[3 * gi + c] = dv;
            if (apply) {
                const double xo = first ? px[c] : as_global(a.x)[3 * gi + c];
                const double Xo = first ? pX[c] : as_global(a.X)[3 * gi + c];
                const double xn = xo + dv;
                as_global(a.x)[3 * gi + c] = xn;
                du[c] = (float)(xn - Xo);
            }
        }
        if (apply) store_global4(a.u + gi, du[0], du[1], du[2], 0.0f);
    }
}

__global__ __launch_bounds__(BLK) void k_refine(const DevMesh* __restrict__ GM, const int32_t* __restrict__ L,
                                                const int32_t* __restrict__ active) {
    Slot sl;
    if (!slot_of(L, active, sl)) return;
    const DevMesh& M = GM[sl.g];
    const int32_t n_free = M.n_free;
    const int32_t* __restrict__ Kp = M.K_ptr;
    const int32_t* __restrict__ Kc = M.K_col;
    const double* __restrict__ Kv = M.K_val;
    const double* __restrict__ delta = M.delta;
    double* __restrict__ r = M.r;
    const int32_t i = sl.lb * BLK + threadIdx.x;
    if (i >= n_free) return;
    double s0 = 0, s1 = 0, s2 = 0;
    csr_row3(Kp, Kc, Kv, delta, i, s0, s1, s2);
    r[3 * i] -= s0;
    r[3 * i + 1] -= s1;
    r[3 * i + 2] -= s2;
}

// ---------------------------------------------------------------------------
// Inexact CMS solve of Sec. 7.2 (selectable instead of the interior back
// substitution).  The condensed interface right-hand side b^b + sum_d Psi_d^T
// b_d^i is what the interior forward solve already produces (the same
// vector), so the interface values x^b are the exact ones; the interiors are
// rebuilt from the subspace of Eq. global_subspace,
//   x_d^i = Phi_d Lambda_d^{-1} Phi_d^T b_d^i + Psi_d x^b,
// with the dense modes read from HBM (FP32 values, FP64 sums), and the whole
// vector is polished by Jacobi sweeps with Chebyshev weights.  b = r (the PD
// residual), x = d (the correction of the iterate).
// ---------------------------------------------------------------------------
constexpr int BLKC = 256;
constexpr int kCmsSlices = 8;          // workgroups per subdomain in k_cms_back

// q_d = Lambda_d^{-1} Phi_d^T b_d^i, `groups` workgroups per subdomain (table
// entry blockIdx.x / groups), one mode per wave (lanes over the rows), to
// cms_q [D][modes][3]
__global__ __launch_bounds__(BLKC) void k_cms_modes(const DevMesh* __restrict__ GM, const int32_t* __restrict__ L,
                                                    const int32_t* __restrict__ active, int32_t groups) {
    const int4 ent = reinterpret_cast<const int4*>(L)[blockIdx.x / groups];
    if (active[ent.x] == 0) return;
    const DevMesh& M = GM[ent.x];
    const int32_t d = ent.y;
    const int32_t r0 = M.sub_off[d], n = M.sub_off[d + 1] - r0;
    const int32_t R = M.cms_modes;
    const float* phi = M.cms_phi + M.cms_phi_off[d];
    const double* rb = M.r + 3 * (size_t)r0;
    const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
    const int32_t k = (int32_t)(blockIdx.x % groups) * (BLKC / 64) + wave;   // this wave's mode
    if (k >= R) return;
    double s0 = 0.0, s1 = 0.0, s2 = 0.0;
#pragma unroll 4
    for (int32_t i = lane; i < n; i += 64) {
        const double f = (double)phi[(size_t)k * n + i];
        s0 += f * rb[3 * i];
        s1 += f * rb[3 * i + 1];
        s2 += f * rb[3 * i + 2];
    }
    s0 = group_sum<64>(s0);
    s1 = group_sum<64>(s1);
    s2 = group_sum<64>(s2);
    if (lane == 0) {
        const double il = (double)M.cms_ilam[(size_t)d * R + k];
        double* q = M.cms_q + 3 * ((size_t)d * R + k);
        q[0] = s0 * il;
        q[1] = s1 * il;
        q[2] = s2 * il;
    }
}

// x^i = Phi q + Psi x^b: kCmsSlices workgroups per subdomain (table entry
// blockIdx.x / kCmsSlices), each a contiguous slice of the rows, one row per
// thread (coalesced column reads of the column-major modes)
__global__ __launch_bounds__(BLKC) void k_cms_back(const DevMesh* __restrict__ GM, const int32_t* __restrict__ L,
                                                   const int32_t* __restrict__ active) {
    extern __shared__ double csm[];
    const int4 ent = reinterpret_cast<const int4*>(L)[blockIdx.x / kCmsSlices];
    if (active[ent.x] == 0) return;
    const DevMesh& M = GM[ent.x];
    const int32_t d = ent.y, slice = blockIdx.x % kCmsSlices;
    const int32_t r0 = M.sub_off[d], n = M.sub_off[d + 1] - r0;
    const int32_t b0 = M.bnd_off[d], nb = M.bnd_off[d + 1] - b0;
    const int32_t R = M.cms_modes;
    const int32_t per = (n + kCmsSlices - 1) / kCmsSlices;
    const int32_t i0 = slice * per, i1 = min(n, i0 + per);
    if (i0 >= i1) return;
    double* XB = csm;                  // [nb][3] interface values
    double* Q = XB + 3 * nb;           // [R][3]
    const int tid = threadIdx.x;
    for (int32_t i = tid; i < 3 * nb; i += BLKC) {
        const int32_t k = i / 3, c = i - 3 * k;
        XB[i] = M.dg[3 * (size_t)(M.bnd[b0 + k] - M.n_int) + c];
    }
    for (int32_t i = tid; i < 3 * R; i += BLKC) Q[i] = M.cms_q[3 * (size_t)d * R + i];
    __syncthreads();
    const float* phi = M.cms_phi + M.cms_phi_off[d];
    const float* psi = M.cms_psi + M.cms_psi_off[d];
    for (int32_t i = i0 + tid; i < i1; i += BLKC) {
        double s0 = 0.0, s1 = 0.0, s2 = 0.0;
#pragma unroll 4
        for (int32_t k = 0; k < R; ++k) {
            const double f = (double)phi[(size_t)k * n + i];
            s0 += f * Q[3 * k];
            s1 += f * Q[3 * k + 1];
            s2 += f * Q[3 * k + 2];
        }
#pragma unroll 8
        for (int32_t j = 0; j < nb; ++j) {
            // the boundary modes (about 100 MB for the shell) are read once
            // per solve: streamed, so they do not evict the interface factor
            // (3.28 -> 3.04 ms/frame; the interior modes, read twice, are not)
            const double f = (double)__builtin_nontemporal_load(psi + (size_t)j * n + i);
            s0 += f * XB[3 * j];
            s1 += f * XB[3 * j + 1];
            s2 += f * XB[3 * j + 2];
        }
        double* dp = M.delta + 3 * (size_t)(r0 + i);
        dp[0] = s0;
        dp[1] = s1;
        dp[2] = s2;
    }
}

// interface rows of the correction: the interface solution
__global__ __launch_bounds__(BLK) void k_cms_iface(const DevMesh* __restrict__ GM, const int32_t* __restrict__ L,
                                                   const int32_t* __restrict__ active) {
    Slot sl;
    if (!slot_of(L, active, sl)) return;
    const DevMesh& M = GM[sl.g];
    const int32_t i = sl.lb * BLK + threadIdx.x;
    if (i < M.n_int || i >= M.n_free) return;
#pragma unroll
    for (int c = 0; c < 3; ++c) M.delta[3 * (size_t)i + c] = M.dg[3 * (size_t)(i - M.n_int) + c];
}

// Jacobi sweep k with the Chebyshev weight omega_k:
//   xhat = x_k + D^{-1} (r - K x_k),  x_{k+1} = omega_k (xhat - x_{k-1}) + x_{k-1}
// buffers: x_k in B[k % 3], x_{k-1} in B[(k + 2) % 3] (x_0 for k = 0, where
// omega = 1), x_{k+1} to B[(k + 1) % 3]; B = {delta, cms_b1, cms_b2}
__global__ __launch_bounds__(BLK) void k_cms_sweep(const DevMesh* __restrict__ GM, const int32_t* __restrict__ L,
                                                   const int32_t* __restrict__ active, int32_t k) {
    Slot sl;
    if (!slot_of(L, active, sl)) return;
    const DevMesh& M = GM[sl.g];
    const int32_t i = sl.lb * BLK + threadIdx.x;
    if (i >= M.n_free) return;
    double* B[3] = {M.delta, M.cms_b1, M.cms_b2};
    const double* xk = B[k % 3];
    const double* xp = (k == 0) ? B[0] : B[(k + 2) % 3];
    double* xn = B[(k + 1) % 3];
    double s0 = 0.0, s1 = 0.0, s2 = 0.0;
    csr_row3(M.K_ptr, M.K_col, M.K_val, xk, i, s0, s1, s2);
    const double id = M.cms_invd[i], om = M.cms_omega[k];
    const double* rr = M.r + 3 * (size_t)i;
    const double h0 = xk[3 * i] + id * (rr[0] - s0);
    const double h1 = xk[3 * i + 1] + id * (rr[1] - s1);
    const double h2 = xk[3 * i + 2] + id * (rr[2] - s2);
    xn[3 * i] = om * (h0 - xp[3 * i]) + xp[3 * i];
    xn[3 * i + 1] = om * (h1 - xp[3 * i + 1]) + xp[3 * i + 1];
    xn[3 * i + 2] = om * (h2 - xp[3 * i + 2]) + xp[3 * i + 2];
}

// the final correction d (in B[sweeps % 3]) to delta; with apply, x += d and
// u = float(x - X); free rows
__global__ __launch_bounds__(BLK) void k_cms_apply(const DevMesh* __restrict__ GM, const int32_t* __restrict__ L,
                                                   const int32_t* __restrict__ active, int32_t sweeps,
                                                   int32_t apply) {
    Slot sl;
    if (!slot_of(L, active, sl)) return;
    const DevMesh& M = GM[sl.g];
    const int32_t i = sl.lb * BLK + threadIdx.x;
    if (i >= M.n_free) return;
    const double* B[3] = {M.delta, M.cms_b1, M.cms_b2};
    const double* dp = B[sweeps % 3] + 3 * (size_t)i;
    const double d0 = dp[0], d1 = dp[1], d2 = dp[2];
    if (sweeps % 3 != 0) {
        M.delta[3 * (size_t)i] = d0;
        M.delta[3 * (size_t)i + 1] = d1;
        M.delta[3 * (size_t)i + 2] = d2;
    }
    if (!apply) return;
    double* xp = M.x + 3 * (size_t)i;
    const double* Xp = M.X + 3 * (size_t)i;
    const double x0 = xp[0] + d0, x1 = xp[1] + d1, x2 = xp[2] + d2;
    xp[0] = x0;
    xp[1] = x1;
    xp[2] = x2;
    store_global4(M.u + i, (float)(x0 - Xp[0]), (float)(x1 - Xp[1]), (float)(x2 - Xp[2]), 0.0f);
}

__global__ __launch_bounds__(BLK) void k_velocity(const DevMesh* __restrict__ GM, const int32_t* __restrict__ L,
                                                  const int32_t* __restrict__ active) {
    Slot sl;
    if (!slot_of(L, active, sl)) return;
    const DevMesh& M = GM[sl.g];
    const int32_t nv = M.nv, n_free = M.n_free;
    const double inv_dt = 1.0 / M.dt;
    const double* __restrict__ x = M.x;
    const double* __restrict__ xprev = M.xprev;
    double* __restrict__ v = M.v;
    uint32_t* flags = M.flags;
    const int32_t i = sl.lb * BLK + threadIdx.x;
    if (i >= nv) return;
    bool bad = false;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const double xv = x[3 * i + c];
        bad |= !isfinite(xv);
        v[3 * i + c] = (i < n_free) ? (xv - xprev[3 * i + c]) * inv_dt : 0.0;
    }
    if (bad) atomicOr(&flags[0], 1u);
}

inline int nblk(int64_t n) { return (int)((n + BLK - 1) / BLK); }

}  // namespace

hipError_t launch_predictor(const LaunchRef& r, hipStream_t s) {
    if (r.nblocks <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_predict, dim3(r.nblocks), dim3(BLK), 0, s, r.G, r.L, r.active);
    return hipGetLastError();
}

hipError_t launch_scatter_colour(const DevMesh& d, const int32_t* list, int32_t count, hipStream_t s) {
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_scatter_colour, dim3((count + BLK - 1) / BLK), dim3(BLK), 0, s, d.trec, d.dbg_T, list, count,
                       d.n_free, d.dbg_b);
    return hipGetLastError();
}

hipError_t launch_local(const LaunchRef& r, hipStream_t s, bool debug) {
    if (r.nblocks <= 0) return hipSuccess;
    if (debug)
        hipLaunchKernelGGL(k_local<true>, dim3(r.nblocks), dim3(LBLK), 0, s, r.G, r.L, r.active);
    else
        hipLaunchKernelGGL(k_local<false>, dim3(r.nblocks), dim3(LBLK), 0, s, r.G, r.L, r.active);
    return hipGetLastError();
}

hipError_t launch_residual(const LaunchRef& r, hipStream_t s) {
    if (r.nblocks <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_residual, dim3(r.nblocks), dim3(BLK), 0, s, r.G, r.L, r.active);
    return hipGetLastError();
}

size_t interior_fwd_lds(int32_t max_n, int32_t max_cint) {
    return sizeof(float) * (2 * (size_t)CHI + 6 * (size_t)max_n + 3 * (size_t)max_cint) + sizeof(int4) * CHD;
}

size_t interior_bwd_lds(int32_t max_n, int32_t max_nb) {
    return sizeof(float) * (2 * (size_t)CHI + 6 * (size_t)max_n + 3 * (size_t)max_nb) + sizeof(int4) * CHD;
}

int32_t interior_chunk_words() { return CHI; }

hipError_t interior_set_lds_limit(size_t bytes) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_interior_fwd),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
    if (e == hipSuccess)
        e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_interior_bwd),
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
    if (e == hipSuccess)
        e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_cms_back),
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
    return e;
}

hipError_t launch_interior_fwd(const LaunchRef& r, size_t lds, hipStream_t s, bool resid) {
    if (r.nblocks <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_interior_fwd, dim3(r.nblocks), dim3(BLKI), lds, s, r.G, r.L, r.active, (int32_t)resid);
    return hipGetLastError();
}

hipError_t launch_coarse(const LaunchRef& r, int32_t kind, int32_t group, hipStream_t s) {
    if (r.nblocks <= 0) return hipSuccess;
    if (group == 64)
        hipLaunchKernelGGL(k_coarse<64>, dim3(r.nblocks), dim3(BLK), 0, s, r.G, r.L, r.active, kind);
    else if (group == 32)
        hipLaunchKernelGGL(k_coarse<32>, dim3(r.nblocks), dim3(BLK), 0, s, r.G, r.L, r.active, kind);
    else
        hipLaunchKernelGGL(k_coarse<16>, dim3(r.nblocks), dim3(BLK), 0, s, r.G, r.L, r.active, kind);
    return hipGetLastError();
}

int32_t coarse_blocks(int32_t ntasks, int32_t group) { return (ntasks + BLK / group - 1) / (BLK / group); }

hipError_t launch_interior_bwd(const LaunchRef& r, size_t lds, hipStream_t s, bool apply, bool keep_delta) {
    if (r.nblocks <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_interior_bwd, dim3(r.nblocks), dim3(BLKI), lds, s, r.G, r.L, r.active,
                       (int32_t)apply, (int32_t)keep_delta);
    return hipGetLastError();
}

hipError_t launch_refine_residual(const LaunchRef& r, hipStream_t s) {
    if (r.nblocks <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_refine, dim3(r.nblocks), dim3(BLK), 0, s, r.G, r.L, r.active);
    return hipGetLastError();
}

hipError_t launch_embed(const float4* rec, const double* x, int32_t n, double* out, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_embed, dim3((n + BLK - 1) / BLK), dim3(BLK), 0, s, rec, x, n, out);
    return hipGetLastError();
}

size_t cms_back_lds(int32_t max_n, int32_t max_nb, int32_t modes) {
    (void)max_n;
    return sizeof(double) * 3 * ((size_t)max_nb + (size_t)modes);
}

hipError_t launch_cms_back(const LaunchRef& r, size_t lds, int32_t modes, hipStream_t s) {
    if (r.nblocks <= 0) return hipSuccess;
    const int32_t groups = (modes + BLKC / 64 - 1) / (BLKC / 64);
    hipLaunchKernelGGL(k_cms_modes, dim3(r.nblocks * groups), dim3(BLKC), 0, s, r.G, r.L, r.active, groups);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_cms_back, dim3(r.nblocks * kCmsSlices), dim3(BLKC), lds, s, r.G, r.L, r.active);
    return hipGetLastError();
}

hipError_t launch_cms_iface(const LaunchRef& r, hipStream_t s) {
    if (r.nblocks <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_cms_iface, dim3(r.nblocks), dim3(BLK), 0, s, r.G, r.L, r.active);
    return hipGetLastError();
}

hipError_t launch_cms_sweep(const LaunchRef& r, int32_t k, hipStream_t s) {
    if (r.nblocks <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_cms_sweep, dim3(r.nblocks), dim3(BLK), 0, s, r.G, r.L, r.active, k);
    return hipGetLastError();
}

hipError_t launch_cms_apply(const LaunchRef& r, int32_t sweeps, bool apply, hipStream_t s) {
    if (r.nblocks <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_cms_apply, dim3(r.nblocks), dim3(BLK), 0, s, r.G, r.L, r.active, sweeps, (int32_t)apply);
    return hipGetLastError();
}

hipError_t launch_velocity(const LaunchRef& r, hipStream_t s) {
    if (r.nblocks <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_velocity, dim3(r.nblocks), dim3(BLK), 0, s, r.G, r.L, r.active);
    return hipGetLastError();
}

int32_t blocks_vertices(int32_t n) { return (n + BLK - 1) / BLK; }
int32_t blocks_tets(int32_t nt) { return (nt + LBLK - 1) / LBLK; }

}  // namespace vh

namespace vh {
namespace {
__global__ __launch_bounds__(BLK) void k_to_user(int32_t nv, const int32_t* __restrict__ perm,
                                                 const double* __restrict__ src,
                                                 double* __restrict__ dst) {
    const int32_t i = blockIdx.x * BLK + threadIdx.x;
    if (i >= nv) return;
    const int32_t u = perm[i];
    dst[3 * u] = src[3 * i];
    dst[3 * u + 1] = src[3 * i + 1];
    dst[3 * u + 2] = src[3 * i + 2];
}

__global__ __launch_bounds__(BLK) void k_from_user(int32_t nv, int32_t n_free,
                                                   const int32_t* __restrict__ perm,
                                                   const double* __restrict__ src,
                                                   const double* __restrict__ X,
                                                   double* __restrict__ dst) {
    const int32_t i = blockIdx.x * BLK + threadIdx.x;
    if (i >= nv) return;
    const int32_t u = perm[i];
#pragma unroll
    for (int c = 0; c < 3; ++c)
        dst[3 * i + c] = (i < n_free) ? src[3 * u + c] : (X ? X[3 * i + c] : 0.0);
}

__global__ __launch_bounds__(BLK) void k_refresh_u(int32_t nv, const double* __restrict__ x,
                                                   const double* __restrict__ X,
                                                   float4* __restrict__ u) {
    const int32_t i = blockIdx.x * BLK + threadIdx.x;
    if (i >= nv) return;
    u[i] = make_float4((float)(x[3 * i] - X[3 * i]), (float)(x[3 * i + 1] - X[3 * i + 1]),
                       (float)(x[3 * i + 2] - X[3 * i + 2]), 0.0f);
}
}  // namespace

hipError_t launch_to_user(int32_t nv, const int32_t* perm, const double* src_int, double* dst_user,
                          hipStream_t s) {
    hipLaunchKernelGGL(k_to_user, dim3(nblk(nv)), dim3(BLK), 0, s, nv, perm, src_int, dst_user);
    return hipGetLastError();
}

hipError_t launch_from_user(int32_t nv, int32_t n_free, const int32_t* perm, const double* src_user,
                            const double* X_or_null, double* dst_int, hipStream_t s) {
    hipLaunchKernelGGL(k_from_user, dim3(nblk(nv)), dim3(BLK), 0, s, nv, n_free, perm, src_user,
                       X_or_null, dst_int);
    return hipGetLastError();
}

hipError_t launch_refresh_u(const DevMesh& m, hipStream_t s) {
    hipLaunchKernelGGL(k_refresh_u, dim3(nblk(m.nv)), dim3(BLK), 0, s, m.nv, m.x, m.X, m.u);
    return hipGetLastError();
}

hipError_t launch_adj_local(const DevMesh* dev_mesh, int32_t nt, const double* xk, const double* xk1,
                            const double* lam, double* gbar, hipStream_t s) {
    if (nt <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_adj_local, dim3(blocks_tets(nt)), dim3(LBLK), 0, s, dev_mesh, xk, xk1, lam, gbar);
    return hipGetLastError();
}

hipError_t launch_adj_gather(const DevMesh* dev_mesh, int32_t n_free, const double* lam, double* xbar,
                             double* ybar, hipStream_t s) {
    if (n_free <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_adj_gather, dim3(nblk(n_free)), dim3(BLK), 0, s, dev_mesh, lam, xbar, ybar);
    return hipGetLastError();
}

hipError_t launch_gn_bd(const DevMesh* dev_mesh, int32_t nt, const double* x, const double* dgam, hipStream_t s) {
    if (nt <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_gn_bd, dim3(blocks_tets(nt)), dim3(LBLK), 0, s, dev_mesh, x, dgam);
    return hipGetLastError();
}

hipError_t launch_gn_av(const DevMesh* dev_mesh, int32_t n_free, const double* v, const double* geo, double* out,
                        hipStream_t s) {
    if (n_free <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_gn_av, dim3(nblk(n_free)), dim3(BLK), 0, s, dev_mesh, v, geo, out);
    return hipGetLastError();
}

hipError_t launch_gn_axpy(int32_t n, double a, const double* x, double* y, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_gn_axpy, dim3(nblk(n)), dim3(BLK), 0, s, n, a, x, y);
    return hipGetLastError();
}

hipError_t launch_gn_xpby(int32_t n, const double* x, double b, double* y, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_gn_xpby, dim3(nblk(n)), dim3(BLK), 0, s, n, x, b, y);
    return hipGetLastError();
}

int32_t gn_dot_blocks() { return 256; }

hipError_t launch_gn_dot(int32_t n, const double* x, const double* y, double* part, hipStream_t s) {
    hipLaunchKernelGGL(k_gn_dot, dim3(gn_dot_blocks()), dim3(BLK), 0, s, n, x, y, part);
    return hipGetLastError();
}

hipError_t launch_adj_frame(int32_t n3, double dt, bool begin, double* xbar, double* vbar, double* xk, double* xn,
                            double* ybar, hipStream_t s) {
    if (n3 <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_adj_frame, dim3(nblk(n3)), dim3(BLK), 0, s, n3, dt, (int32_t)begin, xbar, vbar, xk, xn,
                       ybar);
    return hipGetLastError();
}
}  // namespace vh
