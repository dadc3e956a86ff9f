// Pair forces without any allocation: the same pair kernels as ld_forces,
// with their scratch (packed positions and charges, zero low words, types,
// 64-slot group boxes, the per-split FP64 partial sums) in one file-scope
// device array.  For callers
// that cannot allocate device memory (stream capture, tight serving loops).
#include <cmath>
#include <mutex>

#include "ld_host.h"

namespace {

using namespace ld::host;

constexpr int64_t kStaticMaxN = 65536;
constexpr int kStaticSplit = 4;
constexpr int kStaticBlock = 256;
constexpr size_t kPosBytes = sizeof(float4) * (size_t)kStaticMaxN;
constexpr size_t kTypeBytes = sizeof(int) * (size_t)kStaticMaxN;
constexpr size_t kBoxBytes = sizeof(ld::Box) * (size_t)(kStaticMaxN / ld::kGroup);
constexpr size_t kPartBytes = sizeof(double) * 3 * (size_t)kStaticMaxN * kStaticSplit;
constexpr size_t kStaticBytes = 2 * kPosBytes + kTypeBytes + kBoxBytes + kPartBytes;  // 8.3 MiB

// Each device that runs the entry point holds its own copy until the process
// ends.  Host code never passes this name to a kernel: it uses the device
// address from hipGetSymbolAddress (g_scratch below).
__device__ __align__(256) unsigned char scratch[kStaticBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_scratch[kMaxDevices] = {};

// The device address of `scratch` on the current device (looked up once per
// device, with that device current).
ld_status scratch_ptr(void** out) {
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(LD_EUNSUPPORTED, "device %d", dev);
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_scratch[dev]) {
        void* p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(LD_EHIP, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
        g_scratch[dev] = p;
    }
    *out = g_scratch[dev];
    return LD_OK;
}

// {x, y, z, q_hat} with q_hat = q sqrt(kT l_B) rounded to FP32 (as ld_init),
// zero low words, and the types clamped into [0, T) so that no value can
// index past the pair kernel's type tables.
__global__ __launch_bounds__(kStaticBlock) void k_static_pack(const float* __restrict__ pos,
                                                              const double* __restrict__ q,
                                                              const int* __restrict__ type,
                                                              int n, int T, double qs,
                                                              float4* pos4, float4* lo4,
                                                              int* typ) {
    const int i = blockIdx.x * kStaticBlock + threadIdx.x;
    if (i >= n) return;
    pos4[i] = make_float4(pos[3 * (size_t)i], pos[3 * (size_t)i + 1], pos[3 * (size_t)i + 2],
                          (float)(q[i] * qs));
    lo4[i] = make_float4(0.f, 0.f, 0.f, 0.f);
    typ[i] = min(max(type[i], 0), T - 1);
}

// F[3i + c] = sum over splits (ascending) of the partials, as ld_forces sums.
__global__ __launch_bounds__(kStaticBlock) void k_static_sum(const double* __restrict__ part,
                                                             int splits, int n, double* F) {
    const int i = blockIdx.x * kStaticBlock + threadIdx.x;
    if (i >= n) return;
    double f[3] = {0.0, 0.0, 0.0};
    for (int k = 0; k < splits; ++k)
        for (int c = 0; c < 3; ++c) f[c] += part[((size_t)k * 3 + c) * (size_t)n + i];
    for (int c = 0; c < 3; ++c) F[3 * (size_t)i + c] = f[c];
}

bool on_device(const void* p) {
    if (!p) return false;
    hipPointerAttribute_t a;
    if (hipPointerGetAttributes(&a, p) != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    return a.type == hipMemoryTypeDevice || a.type == hipMemoryTypeManaged;
}

}  // namespace

extern "C" {

ld_status ld_forces_noalloc(int64_t n, const int32_t* type, const double* charge,
                            const float* pos, const ld_params* p, double* F_pair, void* stream) {
    g_err.clear();
    if (n < 2 || n > kStaticMaxN)
        return fail(LD_EINVAL, "n=%lld outside [2, %lld] (the static scratch holds %lld)",
                    (long long)n, (long long)kStaticMaxN, (long long)kStaticMaxN);
    if (!on_device(type) || !on_device(charge) || !on_device(pos) || !on_device(F_pair))
        return fail(LD_EINVAL, "type, charge, pos and F_pair must be device pointers");
    ld_status st = check_params(p);
    if (st != LD_OK) return st;
    void* base = nullptr;
    if ((st = scratch_ptr(&base)) != LD_OK) return st;
    hipStream_t s = (hipStream_t)stream;

    ld::PairTable tab;
    ld::ExtParams ext;
    ld_radius R{};
    R.kind = LD_R_CONST;
    make_tables(*p, R, tab, ext);

    unsigned char* b = (unsigned char*)base;
    float4* pos4 = (float4*)b;
    float4* lo4 = (float4*)(b + kPosBytes);
    int* typ = (int*)(b + 2 * kPosBytes);
    ld::Box* box = (ld::Box*)(b + 2 * kPosBytes + kTypeBytes);
    double* part = (double*)(b + 2 * kPosBytes + kTypeBytes + kBoxBytes);
    const int N = (int)n;
    const dim3 grid((N + kStaticBlock - 1) / kStaticBlock);
    hipLaunchKernelGGL(k_static_pack, grid, dim3(kStaticBlock), 0, s, pos, charge, type, N,
                       p->n_types, std::sqrt(p->kT * p->bjerrum), pos4, lo4, typ);
    HIP_TRY(hipGetLastError());
    HIP_TRY(ld::launch_boxes(pos4, N, box, s));

    ld::PairLaunch L{};
    L.pos = pos4;
    L.lo = lo4;
    L.typ = typ;
    L.box = box;
    L.n = N;
    L.block = kStaticBlock;
    L.j_split = kStaticSplit;
    L.comp = 0;
    L.cull = 1;
    L.Fpart = part;
    L.S = nullptr;
    L.U = nullptr;
    L.nearbits = nullptr;                    // the LJ kernel finds near groups by their boxes
    L.nb_words = 0;
    HIP_TRY(ld::launch_pair(L, tab, s));
    hipLaunchKernelGGL(k_static_sum, grid, dim3(kStaticBlock), 0, s, (const double*)part,
                       kStaticSplit, N, F_pair);
    HIP_TRY(hipGetLastError());
    return LD_OK;
}

}  // extern "C"
