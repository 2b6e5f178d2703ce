// qt_tprod_noalloc: the T-product of qt_tprod with no device allocation, for
// callers that cannot allocate (work under HIP graph capture, serving loops,
// harnesses that forbid hipMalloc).
//
// The workspace (A^, B^, C^ and the fp16 scales, the layout of
// qt_workspace_size) lives in one file-scope device array.  Its device address
// is resolved once per device with hipGetSymbolAddress and only that address
// is handed to kernels: in host code the array's name is a host-side
// stand-in, not a device pointer.  When the plan of p (twiddles, Bluestein
// tables) is not cached yet, the tables are generated into the array behind
// the workspace on every call instead of being allocated.  Nothing in the
// array needs clearing: every workspace region is written before it is read.
#include <mutex>

#include "qt_internal.h"
#include "workspace.h"
#include "../../include/qtprod.h"

namespace {

static __device__ __align__(256) char scratch[QT_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
constexpr size_t kAlign = 256;

std::mutex g_scratch_mutex;
void* g_scratch_ptr[kMaxDevices];   // device address of `scratch` per device

size_t align_up(size_t x) { return (x + kAlign - 1) & ~(kAlign - 1); }

// Device address of the array on the current device (resolved on the first
// call per device, with that device current).
int scratch_address(char** out) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) {
        (void)hipGetLastError();
        return QT_ERR_HIP;
    }
    if (dev < 0 || dev >= kMaxDevices) return QT_ERR_UNSUPPORTED;
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || ptr == nullptr) {
            (void)hipGetLastError();
            return QT_ERR_HIP;
        }
        g_scratch_ptr[dev] = ptr;
    }
    *out = static_cast<char*>(g_scratch_ptr[dev]);
    return QT_OK;
}

// Bytes of the plan tables of p when they have to be generated per call:
// both twiddle tables, then the Bluestein tables if p needs them.
size_t table_bytes(int p) {
    return align_up(sizeof(float2) * (size_t)p) + align_up(sizeof(double2) * (size_t)p) +
           align_up(qt::bluestein_tables_bytes(p));
}

}  // namespace

extern "C" qt_status qt_tprod_noalloc(int m, int n, int s, int p, const void* A, const void* B, void* C,
                                      qt_precision precision, hipStream_t stream) {
    int st = qt::check_tprod(m, n, s, p, A, B, C, precision);
    if (st != QT_OK) return qt::to_status(st);
    if (p > QT_MAX_P) return QT_ERR_UNSUPPORTED;
    const size_t need = align_up(qt_workspace_size(m, n, s, p, precision));
    if (need == 0) return QT_ERR_INVALID_ARG;
    qt::Twiddles tw{};
    const bool cached = qt::find_twiddles(p, &tw);
    const size_t tables = cached ? 0 : table_bytes(p);
    if (need > QT_NOALLOC_SCRATCH_BYTES || tables > QT_NOALLOC_SCRATCH_BYTES - need)
        return QT_ERR_TOO_LARGE;
    char* ws = nullptr;
    st = scratch_address(&ws);
    if (st != QT_OK) return qt::to_status(st);
    if (!cached) {
        char* t = ws + need;
        tw.f32 = reinterpret_cast<float2*>(t);
        t += align_up(sizeof(float2) * (size_t)p);
        tw.f64 = reinterpret_cast<double2*>(t);
        t += align_up(sizeof(double2) * (size_t)p);
        if (qt::launch_twiddles(p, tw, stream) != hipSuccess) return QT_ERR_HIP;
        if (qt::bluestein_tables_bytes(p)) {
            qt::carve_bluestein_tables(p, t, &tw.blue);
            if (qt::launch_bluestein_tables(p, tw.blue, stream) != hipSuccess) return QT_ERR_HIP;
        }
    }
    return qt::to_status(qt::dispatch_tprod(m, n, s, p, A, B, C, precision, ws, stream, &tw));
}
