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

// Optional timing of individual launches (profiling mode only).
void* event_create();
void event_destroy(void* e);
void event_record(void* e, hipStream_t s);
float event_ms(void* start, void* stop);

}  // namespace dev
}  // namespace pe
