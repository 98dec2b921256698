// noalloc.hip -- eifp_step_noalloc: eifp_step's time steps on a caller-owned device
// state, with no device allocation at all, for callers that cannot allocate (code under
// HIP graph capture, tight serving loops, harnesses that forbid hipMalloc).
//
// The state is stepped in place (the transforms run in the caller's buffer, as the
// server's in-place members do).  Everything else a step needs -- the member descriptor,
// the three twiddle tables, the fused pass's per-workgroup partial records and the
// invariant record -- lives in `scratch`, a fixed file-scope device array.  Each device
// the library runs on holds its own copy until the process ends; its device address is
// looked up once per device (hipGetSymbolAddress) and only that address is used in host
// code.  A set-up kernel writes the descriptor and forms the tables (the same formula
// as every other table of the library), so each call depends on nothing a previous call
// left in the array; nothing in it has to start at zero (every partial record is
// written before it is read).  Calls that overlap on one device share the array and race.
#include <hip/hip_runtime.h>

#include <mutex>

#include "engine.h"

using namespace eifp;

namespace {

// 4 MiB: every supported shape fits (the largest need, the FP32 512^3 grid with one
// partial record per fused tile, is about 2.05 MiB).
constexpr size_t kScratchBytes = (size_t)4 << 20;
constexpr size_t kAlign = 256;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};  // device address of `scratch`, per device

// The device address of the current device's copy of `scratch` (looked up on the first
// call on that device, with that device current).
eifp_status scratch_address(void** out) {
    int dev = -1;
    EIFP_HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(EIFP_ERR_DEVICE, "device index %d out of range", dev);
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(EIFP_ERR_DEVICE, "hipGetSymbolAddress(scratch) failed: %s", hipGetErrorString(e));
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return EIFP_OK;
}

size_t align_up(size_t n) { return (n + kAlign - 1) / kAlign * kAlign; }

// The device allocation holding p must reach at least `need` bytes past p (checked on the
// host, so a host pointer or a short buffer is an argument error, not a memory fault).
eifp_status check_device_extent(const void* p, size_t need, const char* what) {
    hipPointerAttribute_t at{};
    const hipError_t ea = hipPointerGetAttributes(&at, p);
    if (ea != hipSuccess || (at.type != hipMemoryTypeDevice && at.type != hipMemoryTypeManaged)) {
        (void)hipGetLastError();
        return fail(EIFP_ERR_INVALID_ARG, "%s is not device memory", what);
    }
    int dev = -1;
    EIFP_HIP_TRY(hipGetDevice(&dev));
    if (at.type == hipMemoryTypeDevice && at.device != dev)
        return fail(EIFP_ERR_INVALID_ARG, "%s is on device %d, the current device is %d", what, at.device, dev);
    hipDeviceptr_t base = nullptr;
    size_t size = 0;
    const hipError_t e = hipMemGetAddressRange(&base, &size, (hipDeviceptr_t)p);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return fail(EIFP_ERR_INVALID_ARG, "%s is not device memory (%s)", what, hipGetErrorString(e));
    }
    const uintptr_t end = (uintptr_t)base + size, q = (uintptr_t)p;
    if (q < (uintptr_t)base || end - q < need)
        return fail(EIFP_ERR_INVALID_ARG, "%s: the allocation holds %zu bytes past the pointer, %zu needed", what,
                    (size_t)(q < end ? end - q : 0), need);
    return EIFP_OK;
}

// Byte offsets of one call's data in `scratch`.
struct Layout {
    size_t desc, inv, twx, twy, twz, partials, end;
};
template <typename T>
Layout layout(int nx, int ny, int nz, int nparts) {
    Layout L;
    size_t o = 0;
    L.desc = o;
    o += align_up(sizeof(DescImage));
    L.inv = o;
    o += align_up(INV_NPART * sizeof(double));
    L.twx = o;
    o += align_up(twiddle_table_bytes<T>(nx));
    L.twy = o;
    o += align_up(twiddle_table_bytes<T>(ny));
    L.twz = o;
    o += align_up(twiddle_table_bytes<T>(nz));
    L.partials = o;
    o += align_up((size_t)nparts * INV_NPART * sizeof(double));
    L.end = o;
    return L;
}

// Set-up: block (i, 0) forms entries of the x table, (i, 1) of y, (i, 2) of z; thread 0
// of block (0, 0) writes the descriptor.
template <typename T>
__global__ void __launch_bounds__(256) k_noalloc_setup(DescImage d, DescImage* __restrict__ desc, cpx<T>* twx, int nx,
                                                       cpx<T>* twy, int ny, cpx<T>* twz, int nz) {
    const int k = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    cpx<T>* tw = blockIdx.y == 0 ? twx : (blockIdx.y == 1 ? twy : twz);
    const int n = blockIdx.y == 0 ? nx : (blockIdx.y == 1 ? ny : nz);
    if (k < n) form_twiddle(tw, n, k);
    if (k == 0 && blockIdx.y == 0) *desc = d;
}

template <typename T>
eifp_status step_noalloc(void* fields, int nx, int ny, int nz, const eifp_domain& dom, double mu, double eps,
                         eifp_precision prec, double tau, long long nsteps, double* inv_out, hipStream_t st) {
    Engine en;  // borrows the tables in `scratch`; owns nothing (never released)
    en.g = Grid3{nx, ny, nz, nx / 2};
    en.prec = prec;
    en.tsize = sizeof(T);
    en.ns = (long long)nx * ny * nz;
    en.nparts = fused_partial_count<T>(AXIS_Y, en.g);
    if (en.nparts <= 0) return fail(EIFP_ERR_UNSUPPORTED_SIZE, "no compiled plan for ny = %d", ny);
    en.nrec = partial_capacity<T>(en.g);
    const Layout L = layout<T>(nx, ny, nz, en.nrec);
    if (L.end > kScratchBytes)
        return fail(EIFP_ERR_UNSUPPORTED_SIZE, "grid %dx%dx%d needs %zu bytes of scratch; the fixed array holds %zu", nx,
                    ny, nz, L.end, kScratchBytes);
    void* base = nullptr;
    eifp_status s;
    if ((s = scratch_address(&base))) return s;
    char* b = (char*)base;
    en.twx = b + L.twx;
    en.twy = b + L.twy;
    en.twz = b + L.twz;
    const DescImage d{fields, fields, (double*)(b + L.partials), inv_out ? inv_out : (double*)(b + L.inv), nullptr,
                      make_params(nx, ny, nz, dom, mu, eps, tau)};
    const int nmax = nx > ny ? (nx > nz ? nx : nz) : (ny > nz ? ny : nz);
    hipLaunchKernelGGL((k_noalloc_setup<T>), dim3((unsigned)((nmax + 255) / 256), 3u), dim3(256), 0, st, d,
                       (DescImage*)(b + L.desc), (cpx<T>*)en.twx, nx, (cpx<T>*)en.twy, ny, (cpx<T>*)en.twz, nz);
    if (hipGetLastError() != hipSuccess) return fail(EIFP_ERR_DEVICE, "set-up kernel launch failed");
    // in place (work == state): one x forward and one x inverse kernel per step; the
    // invariants are reduced on the last step only, and only when asked for
    return en.steps(b + L.desc, 1, nsteps, st, nullptr, inv_out ? nsteps - 1 : nsteps, false);
}

}  // namespace

extern "C" eifp_status eifp_step_noalloc(void* fields, int nx, int ny, int nz, const eifp_domain* dom, double mu,
                                         double eps, eifp_precision prec, double tau, long long nsteps,
                                         double* inv_out, void* hip_stream) {
    clear_error();
    if (!fields || !dom) return fail(EIFP_ERR_INVALID_ARG, "NULL field buffer or domain");
    if (((uintptr_t)fields & 15u) != 0) return fail(EIFP_ERR_INVALID_ARG, "field buffer is not 16-byte aligned");
    if (inv_out && ((uintptr_t)inv_out & 7u) != 0) return fail(EIFP_ERR_INVALID_ARG, "inv_out is not 8-byte aligned");
    eifp_status s;
    if ((s = validate_shape(nx, ny, nz)) || (s = validate_problem(dom, mu, eps)) || (s = validate_tau(tau))) return s;
    if (prec != EIFP_FP64 && prec != EIFP_FP32) return fail(EIFP_ERR_INVALID_ARG, "unknown precision %d", (int)prec);
    if (nsteps < 0) return fail(EIFP_ERR_INVALID_ARG, "nsteps must be >= 0");
    if (nsteps == 0) return EIFP_OK;
    const size_t tsize = prec == EIFP_FP64 ? sizeof(double) : sizeof(float);
    if ((s = check_device_extent(fields, (size_t)6 * nx * ny * nz * tsize, "field buffer")) ||
        (inv_out && (s = check_device_extent(inv_out, INV_NPART * sizeof(double), "inv_out"))))
        return s;
    const hipStream_t st = (hipStream_t)hip_stream;
    return prec == EIFP_FP64 ? step_noalloc<double>(fields, nx, ny, nz, *dom, mu, eps, prec, tau, nsteps, inv_out, st)
                             : step_noalloc<float>(fields, nx, ny, nz, *dom, mu, eps, prec, tau, nsteps, inv_out, st);
}
