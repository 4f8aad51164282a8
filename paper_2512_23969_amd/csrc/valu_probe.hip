// valu_probe.hip -- VALU issue-rate calibration for the roofline of the
// hashing kernels on gfx950 (built by build.py into ./valu_probe; run it
// under rocprofv3 with GRBM_GUI_ACTIVE and SQ_INSTS_VALU to get cycles).
//
// Two kinds of probe, each a grid of 2048 workgroups x 256 lanes (8 waves
// per SIMD) with no memory traffic besides one store per lane:
//   - op probes: 16 independent chains per lane of one instruction, to see
//     which instructions issue faster than one wave64 instruction per 4
//     cycles per SIMD;
//   - unit probes: the library's own SHA-256 and SHA-512 compressions and
//     Keccak-f[1600] permutation, to give the rate (units/s and lane-ops/s)
//     that each instruction mix reaches with no loads, stores or barriers.
// Prints one JSON line per probe.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>

#include "slh_dev.hpp"  // SHA-2 and Keccak device code

namespace {

#define PCHK(x)                                                                   \
  do {                                                                            \
    hipError_t e_ = (x);                                                          \
    if (e_ != hipSuccess) {                                                       \
      std::fprintf(stderr, "HIP error %s at line %d\n", hipGetErrorString(e_), __LINE__); \
      return 1;                                                                   \
    }                                                                             \
  } while (0)

constexpr int kBlocks = 2048, kThreads = 256, kChains = 16;

#define PROBE_BODY(INS) _Pragma("unroll") for (int j = 0; j < kChains; j++) { INS; }

// Instruction probes: OP selects the instruction.
template <int OP>
__global__ __launch_bounds__(kThreads) void k_op(uint32_t* out, int iters, uint32_t seed) {
  uint32_t a[kChains];
#pragma unroll
  for (int j = 0; j < kChains; j++) a[j] = seed * (threadIdx.x + 1) + j * 0x9E3779B9u;
  const uint32_t b = seed ^ blockIdx.x, c = seed + threadIdx.x;
  for (int i = 0; i < iters; i++) {
    if constexpr (OP == 0) PROBE_BODY(asm volatile("v_bitop3_b32 %0, %0, %1, %2 bitop3:0x96" : "+v"(a[j]) : "v"(b), "v"(c)))
    if constexpr (OP == 1) PROBE_BODY(asm volatile("v_xor_b32 %0, %0, %1" : "+v"(a[j]) : "v"(b)))
    if constexpr (OP == 2) PROBE_BODY(asm volatile("v_add_u32 %0, %0, %1" : "+v"(a[j]) : "v"(b)))
    if constexpr (OP == 3) PROBE_BODY(asm volatile("v_lshrrev_b32 %0, 7, %0" : "+v"(a[j])))
    if constexpr (OP == 4) PROBE_BODY(asm volatile("v_lshlrev_b32 %0, 7, %0" : "+v"(a[j])))
    if constexpr (OP == 5) PROBE_BODY(asm volatile("v_alignbit_b32 %0, %0, %1, 7" : "+v"(a[j]) : "v"(b)))
    if constexpr (OP == 6) PROBE_BODY(asm volatile("v_add3_u32 %0, %0, %1, %2" : "+v"(a[j]) : "v"(b), "v"(c)))
    if constexpr (OP == 7) PROBE_BODY(asm volatile("v_perm_b32 %0, %0, %1, %2" : "+v"(a[j]) : "v"(b), "v"(c)))
    if constexpr (OP == 8)
      PROBE_BODY(asm volatile("v_lshl_add_u64 %0, %0, 0, %1"
                              : "+v"(*reinterpret_cast<uint64_t*>(&a[j & 14]))
                              : "v"(*reinterpret_cast<uint64_t*>(&a[(j + 2) & 14]))))
  }
  uint32_t s = 0;
#pragma unroll
  for (int j = 0; j < kChains; j++) s ^= a[j];
  out[blockIdx.x * kThreads + threadIdx.x] = s;
}

// Unit probes.  Each lane chains `iters` units; the next input is derived
// from the previous output so that nothing can be hoisted, and every state
// word differs between lanes so that nothing runs on the scalar unit.
__global__ __launch_bounds__(kThreads) void k_sha256(uint32_t* out, int iters, uint32_t seed) {
  uint32_t st[2][8], w[16];
#pragma unroll
  for (int s = 0; s < 2; s++) {
    slh::sha256_iv(st[s]);
#pragma unroll
    for (int j = 0; j < 8; j++) st[s][j] ^= (seed + threadIdx.x + 977u * blockIdx.x) * (2u * j + 1u + 16u * s);
  }
  for (int i = 0; i < iters; i++) {
#pragma unroll
    for (int s = 0; s < 2; s++) {  // two independent states per lane
#pragma unroll
      for (int j = 0; j < 16; j++) w[j] = st[s][j & 7] + uint32_t(j) + blockIdx.x;
      slh::sha256_compress(st[s], w);
    }
  }
  out[blockIdx.x * kThreads + threadIdx.x] = st[0][0] ^ st[1][3];
}

__global__ __launch_bounds__(kThreads) void k_sha512(uint32_t* out, int iters, uint32_t seed) {
  slh::u64p st[8], w[16];
  slh::sha512_iv(st);
#pragma unroll
  for (int j = 0; j < 8; j++) {
    st[j].lo ^= (seed + threadIdx.x + 977u * blockIdx.x) * (2u * j + 1u);
    st[j].hi ^= (seed + threadIdx.x) * (2u * j + 3u);
  }
  for (int i = 0; i < iters; i++) {
#pragma unroll
    for (int j = 0; j < 16; j++) w[j] = slh::u64p{st[j & 7].hi + blockIdx.x, st[j & 7].lo + uint32_t(j)};
    slh::sha512_compress(st, w);
  }
  out[blockIdx.x * kThreads + threadIdx.x] = st[0].hi ^ st[3].lo;
}

__global__ __launch_bounds__(kThreads) void k_keccak(uint32_t* out, int iters, uint32_t seed) {
  slh::KLane s[25];
#pragma unroll
  for (int i = 0; i < 25; i++)
    s[i] = slh::KLane{(seed + threadIdx.x) * (2u * i + 1u), threadIdx.x + 977u * blockIdx.x * (2u * i + 3u)};
  for (int i = 0; i < iters; i++) slh::keccak_f1600(s);
  out[blockIdx.x * kThreads + threadIdx.x] = s[0].lo ^ s[7].hi;
}

template <typename K>
int time_kernel(K kernel, uint32_t* d, int iters, float* ms) {
  hipEvent_t e0, e1;
  PCHK(hipEventCreate(&e0));
  PCHK(hipEventCreate(&e1));
  hipLaunchKernelGGL(kernel, dim3(kBlocks), dim3(kThreads), 0, 0, d, 4, 1u);  // warm-up
  PCHK(hipGetLastError());
  PCHK(hipDeviceSynchronize());
  PCHK(hipEventRecord(e0));
  hipLaunchKernelGGL(kernel, dim3(kBlocks), dim3(kThreads), 0, 0, d, iters, 2u);
  PCHK(hipEventRecord(e1));
  PCHK(hipEventSynchronize(e1));
  PCHK(hipEventElapsedTime(ms, e0, e1));
  PCHK(hipEventDestroy(e0));
  PCHK(hipEventDestroy(e1));
  return 0;
}

template <int OP>
int run_op(const char* name, uint32_t* d) {
  const int iters = 50000;
  float ms = 0;
  if (time_kernel(k_op<OP>, d, iters, &ms)) return 1;
  const double lane_ops = double(kBlocks) * kThreads * iters * kChains;
  std::printf("{\"probe\": \"op\", \"name\": \"%s\", \"ms\": %.4f, \"lane_ops\": %.6e, \"T_lane_ops_per_s\": %.3f}\n",
              name, ms, lane_ops, lane_ops / (ms * 1e-3) / 1e12);
  std::fflush(stdout);
  return 0;
}

template <typename K>
int run_unit(const char* name, K kernel, int per_iter, int iters, uint32_t* d) {
  float ms = 0;
  if (time_kernel(kernel, d, iters, &ms)) return 1;
  const double units = double(kBlocks) * kThreads * iters * per_iter;
  std::printf("{\"probe\": \"unit\", \"name\": \"%s\", \"ms\": %.4f, \"units\": %.6e, \"units_per_s\": %.6e}\n", name,
              ms, units, units / (ms * 1e-3));
  std::fflush(stdout);
  return 0;
}

}  // namespace

int main() {
  uint32_t* d = nullptr;
  PCHK(hipMalloc(&d, size_t(kBlocks) * kThreads * sizeof(uint32_t)));
  // stop at the first failing launch
  if (run_op<0>("v_bitop3_b32", d) || run_op<1>("v_xor_b32", d) || run_op<2>("v_add_u32", d) ||
      run_op<3>("v_lshrrev_b32", d) || run_op<4>("v_lshlrev_b32", d) || run_op<5>("v_alignbit_b32", d) ||
      run_op<6>("v_add3_u32", d) || run_op<7>("v_perm_b32", d) || run_op<8>("v_lshl_add_u64", d) ||
      run_unit("sha256_compress", k_sha256, 2, 400, d) || run_unit("sha512_compress", k_sha512, 1, 150, d) ||
      run_unit("keccak_f1600", k_keccak, 1, 150, d))
    return 1;
  PCHK(hipFree(d));
  return 0;
}
