// vh_mesh_step_noalloc: the PD step with every work buffer of its kernels in a
// file-scope device array instead of the mesh's own allocations, for callers
// that cannot allocate device memory (code under HIP graph capture, serving
// loops, harnesses that forbid allocation).
//
// The kernels are the step's own; they reach their buffers through a DevMesh
// record, so the variant writes a copy of the mesh's record, with the work
// buffers pointing into the array, at the head of the array and launches the
// mesh's frame with that record.  The array's device address comes from
// hipGetSymbolAddress, once per context (so once per device it is used on),
// with the device current; host code never passes the symbol itself.
#include <algorithm>
#include <type_traits>

#include "runtime.h"

namespace {

// the step's work buffers of one call: force partials, residual, interior and
// interface work vectors, the last correction, interface contribution slots
__device__ __align__(256) unsigned char scratch[VH_NOALLOC_SCRATCH_BYTES];

constexpr size_t kAlign = 256;
size_t round_up(size_t n) { return (n + kAlign - 1) / kAlign * kAlign; }

// dst <- the record passed by value (no host staging, no copy engine)
__global__ void k_put_record(vh::DevMesh rec, vh::DevMesh* dst) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *dst = rec;
}

// zero n 16-byte words
__global__ __launch_bounds__(256) void k_zero16(uint4* p, size_t n) {
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) p[i] = make_uint4(0, 0, 0, 0);
}

// Carves the work buffers of mesh m out of the array at base (a device
// address); returns the bytes used, record included.  With base == 0 only
// counts.
size_t carve(const vh::Plan& P, vh::DevMesh& d, char* base) {
    size_t off = round_up(sizeof(vh::DevMesh));
    auto take = [&](auto** p, size_t count) {
        using T = std::remove_pointer_t<std::remove_reference_t<decltype(*p)>>;
        if (base) *p = reinterpret_cast<T*>(base + off);
        off += round_up(std::max<size_t>(count, 1) * sizeof(T));
    };
    take(&d.part, (size_t)std::max<int32_t>(P.blk_part.back(), 1));
    take(&d.r, (size_t)P.n_free * 3);
    take(&d.zf, (size_t)P.n_int * 3);
    take(&d.rg, (size_t)P.n_gamma * 3);
    take(&d.zg, (size_t)P.n_gamma * 3);
    take(&d.dg, (size_t)P.n_gamma * 3);
    take(&d.delta, (size_t)P.n_free * 3);
    take(&d.cgf, (size_t)P.n_cgf * 3);
    take(&d.cgd, (size_t)P.n_cgd * 3);
    return off;
}

// bytes of the array the mesh's step needs, record included
size_t noalloc_need(const vh_mesh* m) {
    vh::DevMesh d;
    return carve(m->plan, d, nullptr);
}

}  // namespace

namespace vhrt {

int noalloc_init(vh_ctx* ctx) {
    void* p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
        return fail(VH_EDEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    ctx->scratch = p;
    return VH_OK;
}

}  // namespace vhrt

using namespace vhrt;

extern "C" int vh_mesh_step_noalloc(vh_mesh* m, int32_t n_frames, void* stream) {
    VH_TRY(check_solo(m));
    if (n_frames < 0) return fail(VH_EINVAL, "n_frames must be >= 0");
    if (!m->ctx->scratch) return fail(VH_ESTATE, "the context has no scratch address");
    const size_t need = noalloc_need(m);
    if (need > (size_t)VH_NOALLOC_SCRATCH_BYTES)
        return fail(VH_EINVAL, "the mesh needs " + std::to_string(need) + " bytes of step scratch; " +
                                   "vh_mesh_step_noalloc holds " + std::to_string((size_t)VH_NOALLOC_SCRATCH_BYTES));
    if (n_frames == 0) return VH_OK;
    VH_TRY(set_device(m));
    hipStream_t s = static_cast<hipStream_t>(stream);
    char* base = static_cast<char*>(m->ctx->scratch);
    vh::DevMesh rec = m->dm;
    carve(m->plan, rec, base);
    vh::DevMesh* drec = reinterpret_cast<vh::DevMesh*>(base);
    // the work buffers start at zero on every call (the kernels write each
    // before reading it; the clear keeps a call independent of the last one)
    const size_t words = (need - round_up(sizeof(vh::DevMesh))) / 16;
    hipLaunchKernelGGL(k_zero16, dim3(1024), dim3(256), 0, s,
                       reinterpret_cast<uint4*>(base + round_up(sizeof(vh::DevMesh))), words);
    VH_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_put_record, dim3(1), dim3(64), 0, s, rec, drec);
    VH_HIP(hipGetLastError());
    // the mesh's own launch tables, with the record in the array
    for (int32_t f = 0; f < n_frames; ++f) VH_TRY(frame_direct(nullptr, m->ls, s, drec));
    return VH_OK;
}
