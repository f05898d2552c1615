// Thin layer over the HIP runtime calls used by the host runtime.
#pragma once
#include "common.hpp"

namespace pe {
namespace dev {

int device_count();
void set_device(int device);
void* malloc(size_t bytes);              // device memory; throws Error(ST_OOM) on failure
void free(void* p);
void* host_alloc(size_t bytes);          // pinned host memory
void host_free(void* p);
void h2d(void* dst, const void* src, size_t bytes, hipStream_t s);   // asynchronous
void d2h(void* dst, const void* src, size_t bytes, hipStream_t s);   // asynchronous
void d2d(void* dst, const void* src, size_t bytes, hipStream_t s);   // asynchronous
void sync(hipStream_t s);

// A private stream (default priority, not synchronising with the null
// stream), used only to record graphs.
hipStream_t stream_create();
void stream_destroy(hipStream_t s);

// Stream capture into an instantiated graph (returned as an opaque handle),
// and its replay.
void capture_begin(hipStream_t s);
void* capture_end(hipStream_t s);
void capture_abort(hipStream_t s);   // ends a capture after an error, discarding it
void graph_launch(void* exec, hipStream_t s);
void graph_destroy(void* exec);

// Optional timing of individual launches (profiling mode only).
void* event_create();
void event_destroy(void* e);
void event_record(void* e, hipStream_t s);
float event_ms(void* start, void* stop);

}  // namespace dev
}  // namespace pe
