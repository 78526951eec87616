// Vector-ALU throughput probe of libhotref: wavefronts of independent FP32
// or FP64 arithmetic chains, timed with HIP events.  It measures the issue
// ceiling that the force kernels' instruction mix runs against (unpacked
// FP32: the library is built without packed FP32 instructions).
#include <hip/hip_runtime.h>

#include <cstdint>

#include "../../include/hotref.h"

namespace {

constexpr int kBlocks = 8192, kThreads = 256, kIters = 4096, kChains = 16;

// kind 0: FP32 fma; 1: FP32 mul; 2: FP32 add; 3: FP32 fma, mul, add in turn;
// 4: FP32 fma with one reciprocal square root per 16 fma; 5: FP64 fma;
// 6: FP32 fma accumulating into the chain (x = a b + x, the two-operand form)
template <int KIND, typename T>
__global__ void __launch_bounds__(kThreads) k_chains(T* out, T a, T b) {
  T x[kChains];
#pragma unroll
  for (int c = 0; c < kChains; ++c) x[c] = (T)(threadIdx.x + c) * (T)1e-3 + (T)1;
  for (int i = 0; i < kIters; ++i) {
#pragma unroll
    for (int c = 0; c < kChains; ++c) {
      if constexpr (KIND == 0) {
        x[c] = __builtin_fmaf(x[c], a, b);
      } else if constexpr (KIND == 5) {
        x[c] = __builtin_fma(x[c], a, b);
      } else if constexpr (KIND == 1) {
        x[c] = x[c] * a;
      } else if constexpr (KIND == 2) {
        x[c] = x[c] + b;
      } else if constexpr (KIND == 6) {
        x[c] = __builtin_fmaf(a, b, x[c]);
      } else if constexpr (KIND == 3) {
        x[c] = (c % 3 == 0) ? __builtin_fmaf(x[c], a, b) : (c % 3 == 1) ? x[c] * a : x[c] + b;
      } else {
        x[c] = (c == 0) ? __builtin_amdgcn_rsqf(x[c]) : __builtin_fmaf(x[c], a, b);
      }
    }
  }
  T s = 0;
#pragma unroll
  for (int c = 0; c < kChains; ++c) s += x[c];
  out[(size_t)blockIdx.x * kThreads + threadIdx.x] = s;
}

template <int KIND, typename T>
hipError_t launch(void* out, hipStream_t st) {
  k_chains<KIND, T><<<kBlocks, kThreads, 0, st>>>((T*)out, (T)0.999, (T)1e-3);
  return hipGetLastError();
}

hipError_t launch_kind(int kind, void* out, hipStream_t st) {
  switch (kind) {
    case 0: return launch<0, float>(out, st);
    case 1: return launch<1, float>(out, st);
    case 2: return launch<2, float>(out, st);
    case 3: return launch<3, float>(out, st);
    case 4: return launch<4, float>(out, st);
    case 5: return launch<5, double>(out, st);
    case 6: return launch<6, float>(out, st);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace

extern "C" {

size_t hotref_valu_probe_scratch(void) { return sizeof(double) * kBlocks * kThreads; }

hotref_status hotref_valu_probe(int kind, void* scratch, size_t scratch_bytes, int repeats,
                                double* ms, double* wave_instructions) {
  if (kind < 0 || kind > 6 || !scratch || scratch_bytes < hotref_valu_probe_scratch() ||
      repeats < 1 || !ms || !wave_instructions)
    return HOTREF_EINVAL;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  // warm-up: enough launches for the clocks to settle
  for (int r = 0; r < 20 && e == hipSuccess; ++r) e = launch_kind(kind, scratch, nullptr);
  if (e == hipSuccess) e = hipEventRecord(e0, nullptr);
  for (int r = 0; r < repeats && e == hipSuccess; ++r) e = launch_kind(kind, scratch, nullptr);
  if (e == hipSuccess) e = hipEventRecord(e1, nullptr);
  if (e == hipSuccess) e = hipEventSynchronize(e1);
  float t = 0.f;
  if (e == hipSuccess) e = hipEventElapsedTime(&t, e0, e1);
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (e != hipSuccess) return HOTREF_EDEVICE;
  *ms = (double)t / repeats;
  // one chain step is one wave instruction per wavefront
  *wave_instructions = (double)kBlocks * kThreads / 64 * kIters * kChains;
  return HOTREF_OK;
}

}  // extern "C"
