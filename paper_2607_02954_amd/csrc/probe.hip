// Measurement hook: throughput of the atomic adds a particle -> grid transfer
// can be built on, measured on the device of the caller's stream.
//
// The binned transfer sums node contributions in on-chip memory (LDS); which
// LDS add it uses (a float add, or an integer add on fixed-point values) is a
// design choice that this hook measures directly.  The direct transfer uses
// global float atomics, whose rate is measured beside them.
//
// Every LDS probe block owns a 1024-word window; in each iteration the 64
// lanes of a wavefront add to 64 consecutive words (no bank conflicts) at an
// offset that moves by a prime stride, so the adds do not serialise on an
// address.  The global probe adds to scattered words of a caller buffer.
#include <hip/hip_runtime.h>

#include "engine.h"
#include "microcosm.h"

namespace {

constexpr int kProbeThreads = 256;
constexpr int kWords = 1024;

enum ProbeKind : int {
  kLdsF32Rtn = 0,    // LDS float atomicAdd whose result is used
  kLdsF32 = 1,       // LDS float add, result unused
  kLdsU64 = 2,       // LDS 64-bit integer add, result unused
  kLdsU32 = 3        // LDS 32-bit integer add, result unused
};

template <int KIND>
__global__ __launch_bounds__(kProbeThreads) void k_lds_probe(unsigned* sink, int iters) {
  __shared__ __align__(16) unsigned long long s64[kWords];
  float* s32f = (float*)s64;
  unsigned* s32u = (unsigned*)s64;
  for (int i = threadIdx.x; i < kWords; i += kProbeThreads) s64[i] = 0;
  __syncthreads();
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  float acc = 0.f;
  for (int it = 0; it < iters; ++it) {
    const int a = (it * 67 + wv * 256 + lane) & (kWords - 1);
    if constexpr (KIND == kLdsF32Rtn) {
      acc += atomicAdd(s32f + a, 1.0f);
    } else if constexpr (KIND == kLdsF32) {
      atomicAdd(s32f + a, 1.0f);
    } else if constexpr (KIND == kLdsU64) {
      atomicAdd(s64 + a, 1ull);
    } else {
      atomicAdd(s32u + a, 1u);
    }
  }
  __syncthreads();
  // keep every add observable
  if (threadIdx.x == 0) sink[blockIdx.x] = (unsigned)s64[lane] + (unsigned)s32u[3] + __float_as_uint(acc);
}

__global__ __launch_bounds__(kProbeThreads) void k_global_probe(float* buf, unsigned n_words, int iters) {
  // a multiplicative hash scatters each thread's adds over the buffer
  unsigned h = (blockIdx.x * kProbeThreads + threadIdx.x) * 2654435761u;
  for (int it = 0; it < iters; ++it) {
    h = h * 1664525u + 1013904223u;
    unsafeAtomicAdd(buf + (h % n_words), 1.0f);
  }
}

__global__ void k_fill_zero(unsigned* p, size_t n) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) p[i] = 0;
}

sim_status err(sim_status st, const char* msg) { return (sim_status)mc::report_error(st, msg); }

}  // namespace

extern "C" sim_status sim_measure_atomics(void* buf, size_t buf_bytes, void* stream, double* out) {
  if (!buf || !out) return err(SIM_E_INVALID, "NULL argument");
  if (buf_bytes < (64u << 20) || ((uintptr_t)buf % 256))
    return err(SIM_E_INVALID, "the probe buffer must hold 64 MiB and be 256-byte aligned");
  hipStream_t s = (hipStream_t)stream;
  int dev = 0, cus = 0, khz = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      hipDeviceGetAttribute(&khz, hipDeviceAttributeClockRate, dev) != hipSuccess)
    return err(SIM_E_HIP, "device query failed");
  const int blocks = cus * 8;
  const int iters = 4096;
  unsigned* sink = (unsigned*)buf;                         // first 64 KiB: block sinks
  float* gbuf = (float*)((char*)buf + (64 << 10));
  const unsigned gwords = (unsigned)((buf_bytes - (64 << 10)) / 4);
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess) return err(SIM_E_HIP, "hipEventCreate failed");
  if (hipEventCreate(&e1) != hipSuccess) {
    hipEventDestroy(e0);
    return err(SIM_E_HIP, "hipEventCreate failed");
  }
  auto timed = [&](auto launch) -> double {
    launch();                                               // warm-up
    hipEventRecord(e0, s);
    for (int r = 0; r < 5; ++r) launch();
    hipEventRecord(e1, s);
    hipEventSynchronize(e1);
    float ms = 0.f;
    hipEventElapsedTime(&ms, e0, e1);
    return ms * 1e-3 / 5.0;
  };
  const double lane_ops = (double)blocks * kProbeThreads * iters;
  const double clk = (double)khz * 1e3;
  double sec;
  sec = timed([&] { k_lds_probe<kLdsF32Rtn><<<blocks, kProbeThreads, 0, s>>>(sink, iters); });
  out[0] = lane_ops / (sec * clk * cus);
  sec = timed([&] { k_lds_probe<kLdsF32><<<blocks, kProbeThreads, 0, s>>>(sink, iters); });
  out[1] = lane_ops / (sec * clk * cus);
  sec = timed([&] { k_lds_probe<kLdsU64><<<blocks, kProbeThreads, 0, s>>>(sink, iters); });
  out[2] = lane_ops / (sec * clk * cus);
  sec = timed([&] { k_lds_probe<kLdsU32><<<blocks, kProbeThreads, 0, s>>>(sink, iters); });
  out[3] = lane_ops / (sec * clk * cus);
  k_fill_zero<<<1024, 256, 0, s>>>((unsigned*)gbuf, gwords);
  const int giters = 256;
  sec = timed([&] { k_global_probe<<<blocks, kProbeThreads, 0, s>>>(gbuf, gwords, giters); });
  out[4] = (double)blocks * kProbeThreads * giters / (sec * clk);
  out[5] = clk;
  out[6] = cus;
  const hipError_t le = hipGetLastError();
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  if (le != hipSuccess) return err(SIM_E_HIP, hipGetErrorString(le));
  return SIM_OK;
}
