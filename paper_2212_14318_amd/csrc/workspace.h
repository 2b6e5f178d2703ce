// Workspace of an entry point: the caller's buffer, or, when the caller passes
// ws == NULL and ws_bytes == 0, a buffer of `need` bytes taken from the
// stream-ordered allocator on `stream` for the duration of the call (freed on
// the same stream after the call's kernels, so no host synchronisation).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdlib.h>
#include <string.h>

#include "../../include/qtprod.h"

namespace qt {

// An internal status (an int holding a qt_status value) as the ABI's enum.
inline qt_status to_status(int st) { return static_cast<qt_status>(st); }

// Fault injection for tests of the error path: with QTPROD_FAULT=alloc in the
// environment (read once per process), the stream-ordered workspace
// allocation is taken to have failed, so the call returns QT_ERR_ALLOC before
// any launch.  Caller-supplied workspaces are unaffected.
inline bool alloc_fault_injected() {
    static const bool on = [] {
        const char* e = getenv("QTPROD_FAULT");
        return e != nullptr && strcmp(e, "alloc") == 0;
    }();
    return on;
}

// need == 0 (the size query rejected the arguments): run() is called without
// a workspace, so that its own checks return the precise status
// (QT_ERR_UNSUPPORTED or QT_ERR_INVALID_ARG); every run() rejects ws == NULL.
template <typename Run>
qt_status with_workspace(void* ws, size_t ws_bytes, size_t need, hipStream_t stream, Run&& run) {
    if (ws) return to_status(run(ws, ws_bytes));
    if (ws_bytes != 0) return QT_ERR_INVALID_ARG;
    if (need == 0) {
        const int st = run(nullptr, 0);
        return st == QT_OK ? QT_ERR_INVALID_ARG : to_status(st);
    }
    void* tmp = nullptr;
    if (alloc_fault_injected() || hipMallocAsync(&tmp, need, stream) != hipSuccess) {
        (void)hipGetLastError();
        return QT_ERR_ALLOC;
    }
    const int st = run(tmp, need);
    if (hipFreeAsync(tmp, stream) != hipSuccess) {
        (void)hipGetLastError();
        return st == QT_OK ? QT_ERR_HIP : to_status(st);
    }
    return to_status(st);
}

}  // namespace qt
