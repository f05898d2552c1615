// HIP implementation of the device layer.
#include "devapi.hpp"

namespace pe {
namespace dev {

int device_count() {
  int n = 0;
  PE_HIP(hipGetDeviceCount(&n));
  return n;
}

void set_device(int device) { PE_HIP(hipSetDevice(device)); }

void* malloc(size_t bytes) {
  void* p = nullptr;
  if (bytes == 0) bytes = 256;
  hipError_t e = hipMalloc(&p, bytes);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    throw Error(ST_OOM, "hipMalloc of " + std::to_string(bytes) + " bytes failed: " + hipGetErrorString(e));
  }
  return p;
}

void free(void* p) {
  if (p) (void)hipFree(p);
}

void* host_alloc(size_t bytes) {
  void* p = nullptr;
  PE_HIP(hipHostMalloc(&p, bytes ? bytes : 256, hipHostMallocDefault));
  return p;
}

void host_free(void* p) {
  if (p) (void)hipHostFree(p);
}

void h2d(void* dst, const void* src, size_t bytes, hipStream_t s) {
  if (bytes) PE_HIP(hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, s));
}

void d2h(void* dst, const void* src, size_t bytes, hipStream_t s) {
  if (bytes) PE_HIP(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToHost, s));
}

void d2d(void* dst, const void* src, size_t bytes, hipStream_t s) {
  if (bytes) PE_HIP(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToDevice, s));
}

void sync(hipStream_t s) { PE_HIP(hipStreamSynchronize(s)); }

void* event_create() {
  hipEvent_t e;
  PE_HIP(hipEventCreate(&e));
  return (void*)e;
}
void event_destroy(void* e) {
  if (e) (void)hipEventDestroy((hipEvent_t)e);
}
void event_record(void* e, hipStream_t s) { PE_HIP(hipEventRecord((hipEvent_t)e, s)); }
float event_ms(void* a, void* b) {
  float ms = 0.f;
  PE_HIP(hipEventElapsedTime(&ms, (hipEvent_t)a, (hipEvent_t)b));
  return ms;
}

hipStream_t stream_create() {
  hipStream_t s = nullptr;
  PE_HIP(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
  return s;
}

void stream_destroy(hipStream_t s) {
  if (s) (void)hipStreamDestroy(s);
}

void capture_begin(hipStream_t s) { PE_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal)); }

void* capture_end(hipStream_t s) {
  hipGraph_t g = nullptr;
  PE_HIP(hipStreamEndCapture(s, &g));
  hipGraphExec_t x = nullptr;
  const hipError_t e = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  PE_HIP(e);
  return (void*)x;
}

void capture_abort(hipStream_t s) {
  hipGraph_t g = nullptr;
  if (hipStreamEndCapture(s, &g) == hipSuccess && g) (void)hipGraphDestroy(g);
  (void)hipGetLastError();
}

void graph_launch(void* exec, hipStream_t s) { PE_HIP(hipGraphLaunch((hipGraphExec_t)exec, s)); }

void graph_destroy(void* exec) {
  if (exec) (void)hipGraphExecDestroy((hipGraphExec_t)exec);
}

}  // namespace dev
}  // namespace pe
