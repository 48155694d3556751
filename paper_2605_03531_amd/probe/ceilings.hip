// Measured VALU, LDS and matrix-core ceilings of the GPU it runs on (one
// process, one device): the rates the dedispersion kernels' roofline lines are
// taken against. Each kernel runs 512-thread workgroups (8 wavefronts), a grid
// of 2048 workgroups, and loops over blocks of 8 independent instructions of
// one kind (the memory ones followed by a wait), so every wavefront keeps 8 in flight and each CU
// holds 16 or more wavefronts. Rates are wavefront-instructions per clock per
// CU at the device's maximum clock (so a slower sustained clock reads as a
// lower rate) and bytes per clock per CU for the memory instructions.
// Prints one JSON object.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>

namespace {

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
constexpr int kIter = 4096;  // blocks of 8 instructions per wavefront
constexpr int kNt = 512;
constexpr int kGrid = 2048;

// 8 independent ds_read_b64 at an 8-byte lane stride (aligned), then a wait.
__global__ __launch_bounds__(kNt) void k_rd64(uint32_t* out) {
  __shared__ __attribute__((aligned(16))) uint8_t lds[32768];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  for (int i = threadIdx.x; i < 32768 / 4; i += kNt) reinterpret_cast<uint32_t*>(lds)[i] = i;
  __syncthreads();
  // wave w reads bytes [512 w, 512 w + 512) + k * 512 of 4 KiB (offsets below 8 KiB)
  uint32_t addr = (uint32_t)(uintptr_t)lds + 8 * lane + 512 * w;
  uint32_t acc = 0;
  for (int it = 0; it < kIter; ++it) {
    u32x2 r0, r1, r2, r3, r4, r5, r6, r7;
    asm volatile(
        "ds_read_b64 %0, %8 offset:0\n ds_read_b64 %1, %8 offset:512\n"
        "ds_read_b64 %2, %8 offset:1024\n ds_read_b64 %3, %8 offset:1536\n"
        "ds_read_b64 %4, %8 offset:2048\n ds_read_b64 %5, %8 offset:2560\n"
        "ds_read_b64 %6, %8 offset:3072\n ds_read_b64 %7, %8 offset:3584\n"
        "s_waitcnt lgkmcnt(0)\n"
        : "=v"(r0), "=v"(r1), "=v"(r2), "=v"(r3), "=v"(r4), "=v"(r5), "=v"(r6), "=v"(r7)
        : "v"(addr));
    acc += r0.x ^ r1.y ^ r2.x ^ r3.y ^ r4.x ^ r5.y ^ r6.x ^ r7.y;
    addr ^= 8;
  }
  out[blockIdx.x * kNt + threadIdx.x] = acc;
}

// 8 independent ds_read_b128 at a 16-byte lane stride (aligned), then a wait.
__global__ __launch_bounds__(kNt) void k_rd128(uint32_t* out) {
  __shared__ __attribute__((aligned(16))) uint8_t lds[32768];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  for (int i = threadIdx.x; i < 32768 / 4; i += kNt) reinterpret_cast<uint32_t*>(lds)[i] = i;
  __syncthreads();
  // base below 4 KiB, offsets up to 28 KiB: every read ends inside the 32 KiB
  uint32_t addr = (uint32_t)(uintptr_t)lds + 16 * lane + 1024 * (w & 3);
  uint32_t acc = 0;
  for (int it = 0; it < kIter; ++it) {
    u32x4 r0, r1, r2, r3, r4, r5, r6, r7;
    asm volatile(
        "ds_read_b128 %0, %8 offset:0\n ds_read_b128 %1, %8 offset:4096\n"
        "ds_read_b128 %2, %8 offset:8192\n ds_read_b128 %3, %8 offset:12288\n"
        "ds_read_b128 %4, %8 offset:16384\n ds_read_b128 %5, %8 offset:20480\n"
        "ds_read_b128 %6, %8 offset:24576\n ds_read_b128 %7, %8 offset:28672\n"
        "s_waitcnt lgkmcnt(0)\n"
        : "=v"(r0), "=v"(r1), "=v"(r2), "=v"(r3), "=v"(r4), "=v"(r5), "=v"(r6), "=v"(r7)
        : "v"(addr));
    acc += r0.x ^ r1.y ^ r2.z ^ r3.w ^ r4.x ^ r5.y ^ r6.z ^ r7.w;
    addr ^= 16;
  }
  out[blockIdx.x * kNt + threadIdx.x] = acc;
}

// Two 8-byte words 512 bytes apart per lane (ds_read2st64_b64, the form the
// compiler fuses two ds_read_b64 of one base into), 8 independent, then a wait.
__global__ __launch_bounds__(kNt) void k_rd2st64(uint32_t* out) {
  __shared__ __attribute__((aligned(16))) uint8_t lds[32768];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  for (int i = threadIdx.x; i < 32768 / 4; i += kNt) reinterpret_cast<uint32_t*>(lds)[i] = i;
  __syncthreads();
  // base below 4 KiB + 8; reads end below 12 KiB
  const uint32_t a0 = (uint32_t)(uintptr_t)lds + 8 * lane + 512 * w;
  uint32_t acc = 0, x = 0;
  for (int it = 0; it < kIter; ++it) {
    u32x4 r0, r1, r2, r3, r4, r5, r6, r7;
    const uint32_t b0 = a0 + x, b1 = b0 + 1024, b2 = b0 + 2048, b3 = b0 + 3072, b4 = b0 + 4096,
                   b5 = b0 + 5120, b6 = b0 + 6144, b7 = b0 + 7168;
    asm volatile(
        "ds_read2st64_b64 %0, %8 offset0:0 offset1:1\n ds_read2st64_b64 %1, %9 offset0:0 offset1:1\n"
        "ds_read2st64_b64 %2, %10 offset0:0 offset1:1\n ds_read2st64_b64 %3, %11 offset0:0 offset1:1\n"
        "ds_read2st64_b64 %4, %12 offset0:0 offset1:1\n ds_read2st64_b64 %5, %13 offset0:0 offset1:1\n"
        "ds_read2st64_b64 %6, %14 offset0:0 offset1:1\n ds_read2st64_b64 %7, %15 offset0:0 offset1:1\n"
        "s_waitcnt lgkmcnt(0)\n"
        : "=v"(r0), "=v"(r1), "=v"(r2), "=v"(r3), "=v"(r4), "=v"(r5), "=v"(r6), "=v"(r7)
        : "v"(b0), "v"(b1), "v"(b2), "v"(b3), "v"(b4), "v"(b5), "v"(b6), "v"(b7));
    acc += r0.x ^ r1.y ^ r2.z ^ r3.w ^ r4.x ^ r5.y ^ r6.z ^ r7.w;
    x ^= 8;
  }
  out[blockIdx.x * kNt + threadIdx.x] = acc;
}

// Two dwords 4 bytes into each 8-byte lane slot (ds_read2_b32: a 64-bit read
// at 4-byte alignment), 8 independent, then a wait.
__global__ __launch_bounds__(kNt) void k_rd2b32(uint32_t* out) {
  __shared__ __attribute__((aligned(16))) uint8_t lds[32768];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  for (int i = threadIdx.x; i < 32768 / 4; i += kNt) reinterpret_cast<uint32_t*>(lds)[i] = i;
  __syncthreads();
  // base below 4 KiB + 8; reads end below 8 KiB
  const uint32_t a0 = (uint32_t)(uintptr_t)lds + 8 * lane + 512 * w;
  uint32_t acc = 0, x = 0;
  for (int it = 0; it < kIter; ++it) {
    u32x2 r0, r1, r2, r3, r4, r5, r6, r7;
    const uint32_t b0 = a0 + x, b1 = b0 + 512, b2 = b0 + 1024, b3 = b0 + 1536, b4 = b0 + 2048,
                   b5 = b0 + 2560, b6 = b0 + 3072, b7 = b0 + 3584;
    asm volatile(
        "ds_read2_b32 %0, %8 offset0:1 offset1:2\n ds_read2_b32 %1, %9 offset0:1 offset1:2\n"
        "ds_read2_b32 %2, %10 offset0:1 offset1:2\n ds_read2_b32 %3, %11 offset0:1 offset1:2\n"
        "ds_read2_b32 %4, %12 offset0:1 offset1:2\n ds_read2_b32 %5, %13 offset0:1 offset1:2\n"
        "ds_read2_b32 %6, %14 offset0:1 offset1:2\n ds_read2_b32 %7, %15 offset0:1 offset1:2\n"
        "s_waitcnt lgkmcnt(0)\n"
        : "=v"(r0), "=v"(r1), "=v"(r2), "=v"(r3), "=v"(r4), "=v"(r5), "=v"(r6), "=v"(r7)
        : "v"(b0), "v"(b1), "v"(b2), "v"(b3), "v"(b4), "v"(b5), "v"(b6), "v"(b7));
    acc += r0.x ^ r1.y ^ r2.x ^ r3.y ^ r4.x ^ r5.y ^ r6.x ^ r7.y;
    x ^= 8;
  }
  out[blockIdx.x * kNt + threadIdx.x] = acc;
}

// 8 independent ds_write_b64 at an 8-byte lane stride, then a wait.
__global__ __launch_bounds__(kNt) void k_wr64(uint32_t* out) {
  __shared__ __attribute__((aligned(16))) uint8_t lds[32768];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const uint32_t addr = (uint32_t)(uintptr_t)lds + 8 * lane + 512 * w;  // below 4 KiB
  u32x2 v = {(uint32_t)threadIdx.x, 1u};
  for (int it = 0; it < kIter; ++it) {
    asm volatile(
        "ds_write_b64 %0, %1 offset:0\n ds_write_b64 %0, %1 offset:4096\n"
        "ds_write_b64 %0, %1 offset:8192\n ds_write_b64 %0, %1 offset:12288\n"
        "ds_write_b64 %0, %1 offset:16384\n ds_write_b64 %0, %1 offset:20480\n"
        "ds_write_b64 %0, %1 offset:24576\n ds_write_b64 %0, %1 offset:28672\n"
        "s_waitcnt lgkmcnt(0)\n" ::"v"(addr),
        "v"(v)
        : "memory");
    v.y += 1;
  }
  __syncthreads();
  out[blockIdx.x * kNt + threadIdx.x] = reinterpret_cast<uint32_t*>(lds)[threadIdx.x];
}

// 8 independent ds_write_b128 at a 16-byte lane stride, then a wait.
__global__ __launch_bounds__(kNt) void k_wr128(uint32_t* out) {
  __shared__ __attribute__((aligned(16))) uint8_t lds[32768];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const uint32_t addr = (uint32_t)(uintptr_t)lds + 16 * lane + 1024 * (w & 3);
  u32x4 v = {(uint32_t)threadIdx.x, 1u, 2u, 3u};
  for (int it = 0; it < kIter; ++it) {
    asm volatile(
        "ds_write_b128 %0, %1 offset:0\n ds_write_b128 %0, %1 offset:4096\n"
        "ds_write_b128 %0, %1 offset:8192\n ds_write_b128 %0, %1 offset:12288\n"
        "ds_write_b128 %0, %1 offset:16384\n ds_write_b128 %0, %1 offset:20480\n"
        "ds_write_b128 %0, %1 offset:24576\n ds_write_b128 %0, %1 offset:28672\n"
        "s_waitcnt lgkmcnt(0)\n" ::"v"(addr),
        "v"(v)
        : "memory");
    v.y += 1;
  }
  __syncthreads();
  out[blockIdx.x * kNt + threadIdx.x] = reinterpret_cast<uint32_t*>(lds)[threadIdx.x];
}

// 8 independent chains of v_add3_u32 (or v_perm_b32).
template <bool PERM>
__global__ __launch_bounds__(kNt) void k_valu(uint32_t* out) {
  uint32_t a0 = threadIdx.x, a1 = a0 + 1, a2 = a0 + 2, a3 = a0 + 3, a4 = a0 + 4, a5 = a0 + 5,
           a6 = a0 + 6, a7 = a0 + 7;
  const uint32_t b = blockIdx.x, c = 0x0c010c00u + (b & 3);
  for (int it = 0; it < kIter; ++it) {
    if (PERM)
      asm volatile(
          "v_perm_b32 %0, %0, %8, %9\n v_perm_b32 %1, %1, %8, %9\n"
          "v_perm_b32 %2, %2, %8, %9\n v_perm_b32 %3, %3, %8, %9\n"
          "v_perm_b32 %4, %4, %8, %9\n v_perm_b32 %5, %5, %8, %9\n"
          "v_perm_b32 %6, %6, %8, %9\n v_perm_b32 %7, %7, %8, %9\n"
          : "+v"(a0), "+v"(a1), "+v"(a2), "+v"(a3), "+v"(a4), "+v"(a5), "+v"(a6), "+v"(a7)
          : "v"(b), "v"(c));
    else
      asm volatile(
          "v_add3_u32 %0, %0, %8, %9\n v_add3_u32 %1, %1, %8, %9\n"
          "v_add3_u32 %2, %2, %8, %9\n v_add3_u32 %3, %3, %8, %9\n"
          "v_add3_u32 %4, %4, %8, %9\n v_add3_u32 %5, %5, %8, %9\n"
          "v_add3_u32 %6, %6, %8, %9\n v_add3_u32 %7, %7, %8, %9\n"
          : "+v"(a0), "+v"(a1), "+v"(a2), "+v"(a3), "+v"(a4), "+v"(a5), "+v"(a6), "+v"(a7)
          : "v"(b), "v"(c));
  }
  out[blockIdx.x * kNt + threadIdx.x] = a0 ^ a1 ^ a2 ^ a3 ^ a4 ^ a5 ^ a6 ^ a7;
}

// 8 independent accumulator chains of v_mfma_i32_16x16x64_i8 (the matrix
// instruction of the matrix-core dedispersion).
typedef int32_t i32x4 __attribute__((ext_vector_type(4)));
__global__ __launch_bounds__(kNt) void k_mfma(uint32_t* out) {
  const int l = threadIdx.x & 63;
  const i32x4 a = {l, 3 * l, 5 * l, 7 * l}, b = {11 * l, l, 2 * l, 9 * l};
  i32x4 acc[8];
#pragma unroll
  for (int k = 0; k < 8; ++k) acc[k] = i32x4{k, 0, 0, 0};
  for (int it = 0; it < kIter; ++it) {
#pragma unroll
    for (int k = 0; k < 8; ++k) acc[k] = __builtin_amdgcn_mfma_i32_16x16x64_i8(a, b, acc[k], 0, 0, 0);
  }
  i32x4 s = acc[0];
#pragma unroll
  for (int k = 1; k < 8; ++k) s ^= acc[k];
  out[blockIdx.x * kNt + threadIdx.x] = (uint32_t)(s.x ^ s.y ^ s.z ^ s.w);
}

template <typename F>
float time_ms(F f) {
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return -1.f;
  f();
  if (hipDeviceSynchronize() != hipSuccess) return -1.f;
  (void)hipEventRecord(e0);
  for (int r = 0; r < 5; ++r) f();
  (void)hipEventRecord(e1);
  if (hipEventSynchronize(e1) != hipSuccess) return -1.f;
  float ms = 0.f;
  (void)hipEventElapsedTime(&ms, e0, e1);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return ms / 5;
}

}  // namespace

int main() {
  uint32_t* out = nullptr;
  if (hipMalloc(&out, (size_t)kGrid * kNt * 4) != hipSuccess) {
    std::fprintf(stderr, "allocation failed\n");
    return 1;
  }
  int ncu = 0, khz = 0;
  (void)hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, 0);
  (void)hipDeviceGetAttribute(&khz, hipDeviceAttributeClockRate, 0);
  const double ghz = khz / 1e6;
  const double instr = (double)kGrid * kNt / 64 * kIter * 8;  // wavefront-instructions
  struct Row {
    const char* name;
    float ms;
    int bytes;  // per lane per instruction (0: VALU)
  } rows[] = {
      {"ds_read_b64", time_ms([&] { hipLaunchKernelGGL(k_rd64, dim3(kGrid), dim3(kNt), 0, 0, out); }), 8},
      {"ds_read_b128", time_ms([&] { hipLaunchKernelGGL(k_rd128, dim3(kGrid), dim3(kNt), 0, 0, out); }), 16},
      {"ds_read2st64_b64", time_ms([&] { hipLaunchKernelGGL(k_rd2st64, dim3(kGrid), dim3(kNt), 0, 0, out); }), 16},
      {"ds_read2_b32_4byte_aligned", time_ms([&] { hipLaunchKernelGGL(k_rd2b32, dim3(kGrid), dim3(kNt), 0, 0, out); }), 8},
      {"ds_write_b64", time_ms([&] { hipLaunchKernelGGL(k_wr64, dim3(kGrid), dim3(kNt), 0, 0, out); }), 8},
      {"ds_write_b128", time_ms([&] { hipLaunchKernelGGL(k_wr128, dim3(kGrid), dim3(kNt), 0, 0, out); }), 16},
      {"v_add3_u32", time_ms([&] { hipLaunchKernelGGL(k_valu<false>, dim3(kGrid), dim3(kNt), 0, 0, out); }), 0},
      {"v_perm_b32", time_ms([&] { hipLaunchKernelGGL(k_valu<true>, dim3(kGrid), dim3(kNt), 0, 0, out); }), 0},
      {"v_mfma_i32_16x16x64_i8", time_ms([&] { hipLaunchKernelGGL(k_mfma, dim3(kGrid), dim3(kNt), 0, 0, out); }), 0},
  };
  if (hipDeviceSynchronize() != hipSuccess) {
    std::fprintf(stderr, "device error\n");
    return 1;
  }
  std::printf("{\"cus\": %d, \"max_clock_ghz\": %.3f", ncu, ghz);
  for (const Row& r : rows) {
    const double per_clk = instr / (r.ms * 1e-3) / (ncu * ghz * 1e9);
    std::printf(", \"%s\": {\"ms\": %.4f, \"wave_instr_per_clk_cu\": %.4f", r.name, r.ms, per_clk);
    if (r.bytes) std::printf(", \"bytes_per_clk_cu\": %.1f", per_clk * 64 * r.bytes);
    std::printf("}");
  }
  std::printf("}\n");
  (void)hipFree(out);
  return 0;
}
