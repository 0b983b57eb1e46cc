// noalloc.hip -- y = A x without any allocation, for callers that cannot
// allocate device memory (code under HIP graph capture, tight serving loops,
// harnesses that forbid hipMalloc).
//
// The operator kernels need one scratch buffer besides x and y: the
// shared-face partial sums of the brick kernels, read back by the combine
// pass of the same call.  Here it is a file-scope device array of fixed size
// (each GPU the library runs on holds one until the process ends).  Host code
// never passes the array's name to a kernel: its device address is looked up
// once per device with hipGetSymbolAddress, with that device current, and
// only that address is used.
//
// Every slot the combine pass reads is written by the same call's brick
// kernel first, so the buffer needs no clearing and keeps whatever the last
// call left.  Calls that overlap on one GPU (two streams, two host threads)
// share the array and race on it.
#include <mutex>

#include "ctx.hpp"

using namespace mf;

constexpr size_t kScratchBytes = size_t(64) << 20; // 64 MiB per device
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

static void *g_scratch[kMaxDevices];
static std::once_flag g_scratch_once[kMaxDevices];
static hipError_t g_scratch_err[kMaxDevices];

// Device address of this device's scratch array (looked up on first use).
static hipError_t scratch_address(int dev, void **out)
{
    std::call_once(g_scratch_once[dev], [dev] {
        void *p = nullptr;
        g_scratch_err[dev] = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        g_scratch[dev] = p;
    });
    *out = g_scratch[dev];
    return g_scratch_err[dev];
}

extern "C" mf_status mf_operator_apply_noalloc(const mf_mesh *mesh, const mf_operator *op, const void *x, void *y,
                                               mf_stream stream)
{
    KMesh km;
    int64_t nn;
    mf_status st = mesh_to_kmesh(nullptr, mesh, &km, &nn, nullptr);
    if (st) return st;
    if ((st = check_op_desc(nullptr, op))) return st;
    if (!x || !y || x == y) return fail(nullptr, MF_ERR_ARG, "x and y must be distinct non-null device arrays");
    const int comps = op->kind == MF_OSEEN ? 3 : 1;
    const size_t elem = op->precision == MF_FP32 ? sizeof(float) : sizeof(double);
    const size_t need = (size_t)comps * (size_t)face_buffer_elems(km) * elem;
    if (need > kScratchBytes)
        return fail(nullptr, MF_ERR_ARG,
                    "mf_operator_apply_noalloc: the mesh needs %zu bytes of face-buffer scratch, more than the "
                    "%zu bytes the library holds (use mf_operator_apply)",
                    need, kScratchBytes);
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return fail(nullptr, MF_ERR_HIP, "hipGetDevice: %s", hipGetErrorString(e));
    if (dev < 0 || dev >= kMaxDevices) return fail(nullptr, MF_ERR_ARG, "device %d beyond %d", dev, kMaxDevices);
    void *face = nullptr;
    if ((e = scratch_address(dev, &face)) != hipSuccess || !face)
        return fail(nullptr, MF_ERR_HIP, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
    hipStream_t s = (hipStream_t)stream;
    if (op->kind == MF_HEAT)
        e = heat_apply(km, heat_args(op), op->precision == MF_FP32, x, y, face, nullptr, nullptr, s);
    else
        e = oseen_apply(km, oseen_args(op), 0, (const double *)x, (double *)y, face, s);
    if (e != hipSuccess) return fail(nullptr, MF_ERR_HIP, "operator apply: %s", hipGetErrorString(e));
    return MF_OK;
}
