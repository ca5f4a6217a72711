// probe.hip -- measurement utility: the LDS histogram ceiling.
//
// The histogram pass (hist.hip) scatters one LDS atomic per row and
// learner.  This kernel runs the same inner loop, 1,024 threads adding
// 8 bins per 16-byte index load into `learners` LDS histograms of `nb`
// words of 4 or 8 bytes (the pass's two word widths), but reads its bin
// indices from a small table that stays in L2, so that the time it takes is
// the LDS atomic rate of that bin distribution.  It is not part of the
// method.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>

#include "../../include/cwb.h"
#include "../../include/cwb_probe.h"

namespace cwb {
int set_error(int code, const std::string& msg);  // runtime.cpp

namespace {

constexpr int kProbeThreads = 1024;
constexpr int kProbeLearners = 4;
typedef unsigned int p_u32x4 __attribute__((ext_vector_type(4)));

template <typename W>
__global__ void __launch_bounds__(kProbeThreads)
k_lds_probe(const uint16_t* __restrict__ idx, int64_t chunk_mask, int nb, int learners, int steps,
            long long* __restrict__ out) {
  extern __shared__ unsigned long long s_raw[];
  W* s_h = reinterpret_cast<W*>(s_raw);
  const int words = learners * nb;
  for (int i = threadIdx.x; i < words; i += kProbeThreads) s_h[i] = W(0);
  __syncthreads();
  const W v = (W)(threadIdx.x + 1);
  const uint32_t top = (uint32_t)(nb - 1);
  for (int s = 0; s < steps; ++s) {
#pragma unroll
    for (int f = 0; f < kProbeLearners; ++f) {
      if (f < learners) {
        const int64_t c = (((int64_t)blockIdx.x * steps + s) * learners + f) * kProbeThreads +
                          threadIdx.x;
        const p_u32x4 w = *(const __attribute__((address_space(1))) p_u32x4*)(idx + 8 * (c & chunk_mask));
        const uint32_t ws[4] = {w.x, w.y, w.z, w.w};
        W* h = s_h + (size_t)f * nb;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const uint32_t b0 = min(ws[j] & 0xffffu, top), b1 = min(ws[j] >> 16, top);
          __hip_atomic_fetch_add(h + b0, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
          __hip_atomic_fetch_add(h + b1, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        }
      }
    }
  }
  __syncthreads();
  // one checksum per block, so the atomics are not optimised away
  long long acc = 0;
  for (int i = threadIdx.x; i < words; i += kProbeThreads) acc += (long long)s_h[i];
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
  if ((threadIdx.x & 63) == 0) atomicAdd((unsigned long long*)&out[blockIdx.x], (unsigned long long)acc);
}

}  // namespace
}  // namespace cwb

extern "C" int cwb_probe_lds_hist(const uint16_t* idx, int64_t idx_len, int32_t nb, int32_t learners,
                                  int32_t word_bytes, int32_t steps, int32_t blocks, long long* out,
                                  void* stream) {
  if (!idx || !out) return cwb::set_error(CWB_E_INVALID_ARG, "null probe buffer");
  const int64_t chunks = idx_len / 8;  // 16-byte loads of 8 bins: a power of two
  if (idx_len < 8 || idx_len % 8 != 0 || (chunks & (chunks - 1)) != 0 ||
      reinterpret_cast<uintptr_t>(idx) % 16 != 0)
    return cwb::set_error(CWB_E_INVALID_ARG, "probe table: 8 x a power of two bins, 16-byte aligned");
  if (nb < 1 || nb > 8192 || learners < 1 || learners > cwb::kProbeLearners || steps < 1 ||
      blocks < 1 || blocks > 65536 || (word_bytes != 4 && word_bytes != 8))
    return cwb::set_error(CWB_E_INVALID_ARG, "probe sizes out of range");
  const size_t lds = (size_t)learners * nb * word_bytes;
  if (lds > 152 * 1024) return cwb::set_error(CWB_E_INVALID_ARG, "probe histograms above 152 KiB of LDS");
  const hipStream_t st = static_cast<hipStream_t>(stream);
  if (word_bytes == 8) {
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&cwb::k_lds_probe<unsigned long long>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, 152 * 1024);
    hipLaunchKernelGGL(cwb::k_lds_probe<unsigned long long>, dim3(blocks), dim3(cwb::kProbeThreads),
                       lds, st, idx, chunks - 1, nb, learners, steps, out);
  } else {
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&cwb::k_lds_probe<uint32_t>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, 152 * 1024);
    hipLaunchKernelGGL(cwb::k_lds_probe<uint32_t>, dim3(blocks), dim3(cwb::kProbeThreads), lds, st,
                       idx, chunks - 1, nb, learners, steps, out);
  }
  const hipError_t e = hipGetLastError();
  return e == hipSuccess ? CWB_OK : cwb::set_error(CWB_E_DEVICE, std::string("probe launch: ") + hipGetErrorString(e));
}
