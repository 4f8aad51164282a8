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
//   - variant probes: the same units built from other instruction choices
//     (the code variants a kernel could be compiled with), to check that the
//     library's choice is the fastest: SHA-256 with v_bfi / v_xor instead of
//     v_bitop3, SHA-256 with v_add_u32 pairs instead of v_add3_u32, SHA-512
//     with carry pairs instead of v_lshl_add_u64, Keccak-f with theta's
//     one-bit rotate built from dual-rate operations instead of v_alignbit.
//   - occupancy probes: the SHA-256 compression with one or two independent
//     states per lane at 1, 2 and 3 waves per SIMD (256, 512 and 768
//     workgroups of 256 lanes), and SHA-512 and Keccak-f at one wave per
//     SIMD, to see what issue rate a wave sustains with few or no other
//     waves beside it (the verification kernel's situation at batch 4096:
//     one wave per SIMD).
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

// Occupancy probes: S independent SHA-256 states per lane.
template <int S>
__global__ __launch_bounds__(kThreads) void k_sha256_states(uint32_t* out, int iters, uint32_t seed) {
  uint32_t st[S][8], w[16];
#pragma unroll
  for (int s = 0; s < S; s++) {
    slh::sha256_iv(st[s]);
#pragma unroll
    for (int j = 0; j < 8; j++) st[s][j] ^= (seed + threadIdx.x + 977u * blockIdx.x) * (2u * j + 1u + 16u * s);
  }
  for (int i = 0; i < iters; i++) {
#pragma unroll
    for (int s = 0; s < S; s++) {
#pragma unroll
      for (int j = 0; j < 16; j++) w[j] = st[s][j & 7] + uint32_t(j) + blockIdx.x;
      slh::sha256_compress(st[s], w);
    }
  }
  uint32_t r = 0;
#pragma unroll
  for (int s = 0; s < S; s++) r ^= st[s][s & 7];
  out[blockIdx.x * kThreads + threadIdx.x] = r;
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

// ---------------------------------------------------------------- variants
// SHA-256 compression with selectable instruction choices.  ADDS 1: every
// sum as v_add_u32 pairs; LOGIC 1: Ch = v_bfi, Maj = v_xor + v_bfi, the
// three-input XORs as two v_xor (what a target without v_bitop3 has).
template <int ADDS>
__device__ __forceinline__ uint32_t vadd(uint32_t a, uint32_t b) {
  if constexpr (ADDS) {
    uint32_t r;
    asm("v_add_u32 %0, %1, %2" : "=v"(r) : "v"(a), "v"(b));
    return r;
  } else {
    return a + b;
  }
}
template <int LOGIC>
__device__ __forceinline__ uint32_t vxor3(uint32_t a, uint32_t b, uint32_t c) {
  if constexpr (LOGIC) {
    uint32_t t, r;
    asm("v_xor_b32 %0, %1, %2" : "=v"(t) : "v"(a), "v"(b));
    asm("v_xor_b32 %0, %1, %2" : "=v"(r) : "v"(t), "v"(c));
    return r;
  } else {
    return slh::xor3(a, b, c);
  }
}
template <int LOGIC>
__device__ __forceinline__ uint32_t vch(uint32_t e, uint32_t f, uint32_t g) {
  if constexpr (LOGIC) {
    uint32_t r;
    asm("v_bfi_b32 %0, %1, %2, %3" : "=v"(r) : "v"(e), "v"(f), "v"(g));
    return r;
  } else {
    return slh::ch32(e, f, g);
  }
}
template <int LOGIC>
__device__ __forceinline__ uint32_t vmaj(uint32_t a, uint32_t b, uint32_t c) {
  if constexpr (LOGIC) {
    uint32_t t, r;  // majority = (a ^ b) ? c : b
    asm("v_xor_b32 %0, %1, %2" : "=v"(t) : "v"(a), "v"(b));
    asm("v_bfi_b32 %0, %1, %2, %3" : "=v"(r) : "v"(t), "v"(c), "v"(b));
    return r;
  } else {
    return slh::maj32(a, b, c);
  }
}
template <int ADDS, int LOGIC>
__device__ __forceinline__ void sha256_variant(uint32_t st[8], uint32_t w[16]) {
  constexpr slh::K256Table K = slh::k256();
  auto rot = [](uint32_t x, uint32_t r) { return __builtin_amdgcn_alignbit(x, x, r); };
  uint32_t a = st[0], b = st[1], c = st[2], d = st[3], e = st[4], f = st[5], g = st[6], h = st[7];
#pragma unroll
  for (int i = 0; i < 64; i++) {
    if (i >= 16) {
      const uint32_t x15 = w[(i + 1) & 15], x2 = w[(i + 14) & 15];
      const uint32_t s0 = vxor3<LOGIC>(rot(x15, 7), rot(x15, 18), x15 >> 3);
      const uint32_t s1 = vxor3<LOGIC>(rot(x2, 17), rot(x2, 19), x2 >> 10);
      w[i & 15] = vadd<ADDS>(vadd<ADDS>(w[i & 15], s0), vadd<ADDS>(w[(i + 9) & 15], s1));
    }
    const uint32_t S1 = vxor3<LOGIC>(rot(e, 6), rot(e, 11), rot(e, 25));
    const uint32_t S0 = vxor3<LOGIC>(rot(a, 2), rot(a, 13), rot(a, 22));
    const uint32_t t1 = vadd<ADDS>(vadd<ADDS>(h, vadd<ADDS>(K.v[i], w[i & 15])), vadd<ADDS>(S1, vch<LOGIC>(e, f, g)));
    const uint32_t t2 = vadd<ADDS>(S0, vmaj<LOGIC>(a, b, c));
    h = g; g = f; f = e; e = vadd<ADDS>(d, t1); d = c; c = b; b = a; a = vadd<ADDS>(t1, t2);
  }
  st[0] += a; st[1] += b; st[2] += c; st[3] += d; st[4] += e; st[5] += f; st[6] += g; st[7] += h;
}
template <int ADDS, int LOGIC>
__global__ __launch_bounds__(kThreads) void k_sha256_variant(uint32_t* out, int iters, uint32_t seed) {
  uint32_t st[2][8], w[16];
#pragma unroll
  for (int s = 0; s < 2; s++) {
    slh::sha256_iv(st[s]);
#pragma unroll
    for (int j = 0; j < 8; j++) st[s][j] ^= (seed + threadIdx.x + 977u * blockIdx.x) * (2u * j + 1u + 16u * s);
  }
  for (int i = 0; i < iters; i++) {
#pragma unroll
    for (int s = 0; s < 2; s++) {
#pragma unroll
      for (int j = 0; j < 16; j++) w[j] = st[s][j & 7] + uint32_t(j) + blockIdx.x;
      sha256_variant<ADDS, LOGIC>(st[s], w);
    }
  }
  out[blockIdx.x * kThreads + threadIdx.x] = st[0][0] ^ st[1][3];
}

// SHA-512 with every 64-bit add as a v_add_co_u32 / v_addc_co_u32 pair.
__device__ __forceinline__ uint64_t add64_carry(uint64_t a, uint64_t b) {
  uint32_t lo, hi;
  asm("v_add_co_u32 %0, vcc, %2, %3\n\tv_addc_co_u32 %1, vcc, %4, %5, vcc"
      : "=&v"(lo), "=v"(hi)
      : "v"(uint32_t(a)), "v"(uint32_t(b)), "v"(uint32_t(a >> 32)), "v"(uint32_t(b >> 32))
      : "vcc");
  return slh::pair64(hi, lo);
}
__device__ __forceinline__ void sha512_carry(slh::u64p st[8], uint64_t w[16]) {
  using slh::rot64;
  using slh::xor3_u64;
  uint64_t a = slh::to64(st[0]), b = slh::to64(st[1]), c = slh::to64(st[2]), d = slh::to64(st[3]);
  uint64_t e = slh::to64(st[4]), f = slh::to64(st[5]), g = slh::to64(st[6]), h = slh::to64(st[7]);
#pragma unroll 1
  for (int r = 0; r < 80; r += 16) {
#pragma unroll
    for (int i = 0; i < 16; i++) {
      if (r > 0) {
        const uint64_t x15 = w[(i + 1) & 15], x2 = w[(i + 14) & 15];
        const uint64_t s0 = xor3_u64(rot64<1>(x15), rot64<8>(x15), x15 >> 7);
        const uint64_t s1 = xor3_u64(rot64<19>(x2), rot64<61>(x2), x2 >> 6);
        w[i] = add64_carry(add64_carry(w[i], s0), add64_carry(w[(i + 9) & 15], s1));
      }
      const uint64_t S1 = xor3_u64(rot64<14>(e), rot64<18>(e), rot64<41>(e));
      const uint64_t S0 = xor3_u64(rot64<28>(a), rot64<34>(a), rot64<39>(a));
      const uint64_t t1 = add64_carry(add64_carry(h, add64_carry(slh::kK512[r + i], w[i])),
                                      add64_carry(S1, slh::ch_u64(e, f, g)));
      const uint64_t t2 = add64_carry(S0, slh::maj_u64(a, b, c));
      h = g; g = f; f = e; e = add64_carry(d, t1); d = c; c = b; b = a; a = add64_carry(t1, t2);
    }
  }
  st[0] = slh::mk64(add64_carry(slh::to64(st[0]), a)); st[1] = slh::mk64(add64_carry(slh::to64(st[1]), b));
  st[2] = slh::mk64(add64_carry(slh::to64(st[2]), c)); st[3] = slh::mk64(add64_carry(slh::to64(st[3]), d));
  st[4] = slh::mk64(add64_carry(slh::to64(st[4]), e)); st[5] = slh::mk64(add64_carry(slh::to64(st[5]), f));
  st[6] = slh::mk64(add64_carry(slh::to64(st[6]), g)); st[7] = slh::mk64(add64_carry(slh::to64(st[7]), h));
}
__global__ __launch_bounds__(kThreads) void k_sha512_carry(uint32_t* out, int iters, uint32_t seed) {
  slh::u64p st[8];
  uint64_t w[16];
  slh::sha512_iv(st);
#pragma unroll
  for (int j = 0; j < 8; j++) {
    st[j].lo ^= (seed + threadIdx.x + 977u * blockIdx.x) * (2u * j + 1u);
    st[j].hi ^= (seed + threadIdx.x) * (2u * j + 3u);
  }
  for (int i = 0; i < iters; i++) {
#pragma unroll
    for (int j = 0; j < 16; j++) w[j] = slh::pair64(st[j & 7].hi + blockIdx.x, st[j & 7].lo + uint32_t(j));
    sha512_carry(st, w);
  }
  out[blockIdx.x * kThreads + threadIdx.x] = st[0].hi ^ st[3].lo;
}

// Keccak-f whose theta builds rotl1(C) from v_add_u32 (C + C), v_lshrrev and
// a three-input XOR instead of two v_alignbit per column.
__device__ __forceinline__ void keccak_round_fast_theta(slh::KLane s[25], uint64_t rc) {
  using slh::KLane;
  KLane C[5];
#pragma unroll
  for (int x = 0; x < 5; x++) C[x] = slh::kxor3(slh::kxor3(s[x], s[x + 5], s[x + 10]), s[x + 15], s[x + 20]);
  KLane D[5];
#pragma unroll
  for (int x = 0; x < 5; x++) {
    const KLane c = C[(x + 1) % 5], q = C[(x + 4) % 5];
    D[x] = KLane{slh::xor3(q.lo, vadd<1>(c.lo, c.lo), c.hi >> 31), slh::xor3(q.hi, vadd<1>(c.hi, c.hi), c.lo >> 31)};
  }
  KLane B[25];
#define PROBE_KRP(x, y, r) \
  B[(y) + 5 * ((2 * (x) + 3 * (y)) % 5)] = slh::krotl<r>(KLane{s[(x) + 5 * (y)].lo ^ D[x].lo, s[(x) + 5 * (y)].hi ^ D[x].hi});
  PROBE_KRP(0, 0, 0) PROBE_KRP(1, 0, 1) PROBE_KRP(2, 0, 62) PROBE_KRP(3, 0, 28) PROBE_KRP(4, 0, 27)
  PROBE_KRP(0, 1, 36) PROBE_KRP(1, 1, 44) PROBE_KRP(2, 1, 6) PROBE_KRP(3, 1, 55) PROBE_KRP(4, 1, 20)
  PROBE_KRP(0, 2, 3) PROBE_KRP(1, 2, 10) PROBE_KRP(2, 2, 43) PROBE_KRP(3, 2, 25) PROBE_KRP(4, 2, 39)
  PROBE_KRP(0, 3, 41) PROBE_KRP(1, 3, 45) PROBE_KRP(2, 3, 15) PROBE_KRP(3, 3, 21) PROBE_KRP(4, 3, 8)
  PROBE_KRP(0, 4, 18) PROBE_KRP(1, 4, 2) PROBE_KRP(2, 4, 61) PROBE_KRP(3, 4, 56) PROBE_KRP(4, 4, 14)
#undef PROBE_KRP
#pragma unroll
  for (int y = 0; y < 5; y++)
#pragma unroll
    for (int x = 0; x < 5; x++)
      s[x + 5 * y] = slh::kchi(B[x + 5 * y], B[(x + 1) % 5 + 5 * y], B[(x + 2) % 5 + 5 * y]);
  s[0].lo ^= uint32_t(rc);
  s[0].hi ^= uint32_t(rc >> 32);
}
__global__ __launch_bounds__(kThreads) void k_keccak_fast_theta(uint32_t* out, int iters, uint32_t seed) {
  slh::KLane s[25];
#pragma unroll
  for (int i = 0; i < 25; i++)
    s[i] = slh::KLane{(seed + threadIdx.x) * (2u * i + 1u), threadIdx.x + 977u * blockIdx.x * (2u * i + 3u)};
  for (int i = 0; i < iters; i++) {
#pragma unroll 1
    for (int r = 0; r < 24; r += 2) {
      keccak_round_fast_theta(s, slh::kKeccakRC[r]);
      keccak_round_fast_theta(s, slh::kKeccakRC[r + 1]);
    }
  }
  out[blockIdx.x * kThreads + threadIdx.x] = s[0].lo ^ s[7].hi;
}

// `blocks` workgroups of kThreads lanes (at most kBlocks: `d` holds one word
// per lane of kBlocks workgroups).
template <typename K>
int time_kernel(K kernel, uint32_t* d, int iters, float* ms, int blocks = kBlocks) {
  if (blocks < 1 || blocks > kBlocks) return 1;
  hipEvent_t e0, e1;
  PCHK(hipEventCreate(&e0));
  PCHK(hipEventCreate(&e1));
  hipLaunchKernelGGL(kernel, dim3(blocks), dim3(kThreads), 0, 0, d, 4, 1u);  // warm-up
  PCHK(hipGetLastError());
  PCHK(hipDeviceSynchronize());
  PCHK(hipEventRecord(e0));
  hipLaunchKernelGGL(kernel, dim3(blocks), dim3(kThreads), 0, 0, d, iters, 2u);
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

template <typename K>
int run_occupancy(const char* name, K kernel, int states, int blocks, int iters, uint32_t* d) {
  float ms = 0;
  if (time_kernel(kernel, d, iters, &ms, blocks)) return 1;
  const double units = double(blocks) * kThreads * iters * states;
  std::printf("{\"probe\": \"occupancy\", \"name\": \"%s\", \"waves_per_simd\": %d, \"states_per_lane\": %d, "
              "\"ms\": %.4f, \"units\": %.6e, \"units_per_s\": %.6e}\n",
              name, blocks / 256, states, ms, units, units / (ms * 1e-3));
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
      run_unit("keccak_f1600", k_keccak, 1, 150, d) ||
      run_unit("variant sha256 add pairs", k_sha256_variant<1, 0>, 2, 400, d) ||
      run_unit("variant sha256 bfi/xor", k_sha256_variant<0, 1>, 2, 400, d) ||
      run_unit("variant sha256 reference", k_sha256_variant<0, 0>, 2, 400, d) ||
      run_unit("variant sha512 carry pairs", k_sha512_carry, 1, 150, d) ||
      run_unit("variant keccak theta dual-rate", k_keccak_fast_theta, 1, 150, d) ||
      run_occupancy("sha256 1 state", k_sha256_states<1>, 1, 256, 2000, d) ||
      run_occupancy("sha256 1 state", k_sha256_states<1>, 1, 512, 2000, d) ||
      run_occupancy("sha256 1 state", k_sha256_states<1>, 1, 768, 2000, d) ||
      run_occupancy("sha256 2 states", k_sha256_states<2>, 2, 256, 1000, d) ||
      run_occupancy("sha256 2 states", k_sha256_states<2>, 2, 512, 1000, d) ||
      run_occupancy("sha256 1 state", k_sha256_states<1>, 1, 2048, 400, d) ||
      run_occupancy("sha512 1 state", k_sha512, 1, 256, 1000, d) ||
      run_occupancy("keccak 1 state", k_keccak, 1, 256, 1000, d))
    return 1;
  PCHK(hipFree(d));
  return 0;
}
