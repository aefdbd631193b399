// Host helpers shared by the entry points.
#pragma once
#include "dcstedc.h"
#include <hip/hip_runtime.h>

#include <cstddef>
#include <vector>

dc_opts dc_resolve_opts(const dc_opts* opt);
hipError_t dc_fill_int(int* p, int n, int v, hipStream_t s);
// Copies nbytes (<= 1024) from host memory into device memory through a
// kernel argument (graph-safe, no host pointer is retained).
hipError_t dc_write_blob(void* dst, const void* src, int nbytes, hipStream_t s);
// Library-owned status word of a stream (created on first use).
hipError_t dc_status_word(hipStream_t s, int** out);

// Device-to-host reads that sit between kernels on the critical path (sizes
// and ranks the host needs before its next launch): the bytes go through a
// pinned per-thread buffer, so the copies are asynchronous, and the wait polls
// the stream instead of sleeping in the runtime, whose wake-up costs several
// hundred microseconds.  On return every dst holds its bytes.
struct DcRead {
    void* dst;
    const void* src;
    size_t n;
};
hipError_t dc_readback(const std::vector<DcRead>& reads, hipStream_t s);

// Host-to-device upload of small host data (layouts, task lists) without a
// host wait: the bytes are copied into a pinned per-thread chunk, which is
// reused only once an event recorded behind its copy has completed.
hipError_t dc_upload(void* dst, const void* src, size_t n, hipStream_t s);
