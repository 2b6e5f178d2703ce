// Workspace of an entry point: the caller's buffer, or, when the caller passes
// ws == NULL and ws_bytes == 0, a buffer of `need` bytes taken from the
// stream-ordered allocator on `stream` for the duration of the call (freed on
// the same stream after the call's kernels, so no host synchronisation).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>

#include "../../include/qtprod.h"

namespace qt {

// need == 0 (the size query rejected the arguments): run() is called without
// a workspace, so that its own checks return the precise status
// (QT_ERR_UNSUPPORTED or QT_ERR_INVALID_ARG); every run() rejects ws == NULL.
template <typename Run>
int with_workspace(void* ws, size_t ws_bytes, size_t need, hipStream_t stream, Run&& run) {
    if (ws) return run(ws, ws_bytes);
    if (ws_bytes != 0) return QT_ERR_INVALID_ARG;
    if (need == 0) {
        const int st = run(nullptr, 0);
        return st == QT_OK ? QT_ERR_INVALID_ARG : st;
    }
    void* tmp = nullptr;
    if (hipMallocAsync(&tmp, need, stream) != hipSuccess) {
        (void)hipGetLastError();
        return QT_ERR_ALLOC;
    }
    const int st = run(tmp, need);
    if (hipFreeAsync(tmp, stream) != hipSuccess) {
        (void)hipGetLastError();
        return st == QT_OK ? QT_ERR_HIP : st;
    }
    return st;
}

}  // namespace qt
