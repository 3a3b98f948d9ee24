// lds_atomics.hip -- LDS atomic-add throughput of one gfx950 chip.
//
// Every workgroup (256 threads) keeps a 16 KiB LDS array; each lane adds to
// an address chosen by the access pattern, `iters` times, with the base
// offset rotating over 8 slots so that consecutive adds do not hit the same
// address.  The adds go through pointers in the local address space, so
// every op is one ds_add_* instruction (a generic pointer can turn a float
// add into a compare-and-swap loop).  Printed: lane-operations per second,
// per clock per CU (256 CUs, 2.4 GHz), and clocks per wave instruction per
// CU, the figures behind the splat's LDS-atomic roofline.
//
//   hipcc --offload-arch=gfx950 -O3 -munsafe-fp-atomics \
//         -Xclang -target-feature -Xclang -packed-fp32-ops \
//         -o lds_atomics lds_atomics.hip && ./lds_atomics
#include <hip/hip_runtime.h>

#include <cstdio>

constexpr int kWords = 4096;          // 32-bit words of the LDS array

typedef __attribute__((address_space(3))) float lds_f32;
typedef __attribute__((address_space(3))) unsigned int lds_u32;
typedef __attribute__((address_space(3))) unsigned long long lds_u64;

// op 0: float add, 1: 32-bit integer add, 2: 64-bit integer add
// pattern 0: one address per lane; 1: two lanes per address;
//         2: three interleaved channels (12-byte stride for 32-bit words,
//            24-byte for 64-bit ones);
//         3: every other lane active, one address per active lane;
//         4: scattered addresses (a hash of lane and iteration);
//         5: lanes 0..31 active (one address per lane);
//         6: lanes 0..15 active;
//         7: four lanes per 8-byte word apart (stride 4 words, 8 lanes of
//            each 16 in one row of a planar tile)
template <int OP, int PAT>
__global__ __launch_bounds__(256) void k_lds(float* out, int iters) {
  __shared__ unsigned int s[kWords];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  for (int i = tid; i < kWords; i += 256) s[i] = 0u;
  __syncthreads();
  const int nw = OP == 2 ? kWords / 2 : kWords;   // elements of the op's width
  lds_f32* sf = (lds_f32*)(s);
  lds_u32* su = (lds_u32*)(s);
  lds_u64* s64 = (lds_u64*)(s);
  int a;
  if (PAT == 0 || PAT == 3 || PAT == 5 || PAT == 6) a = wave * 64 + lane;
  else if (PAT == 7) a = wave * 256 + 4 * lane;
  else if (PAT == 1) a = wave * 64 + lane / 2;
  else a = wave * 192 + 3 * lane;
  const bool on = PAT == 3 ? (lane & 1) == 0 : PAT == 5 ? lane < 32 : PAT == 6 ? lane < 16 : true;
  for (int it = 0; it < iters; ++it) {
    int e;
    if (PAT == 4) {
      unsigned int hsh = (unsigned int)(tid * 0x9E3779B1u) ^ (unsigned int)(it * 0x85EBCA77u);
      hsh ^= hsh >> 15;
      e = (int)(hsh % (unsigned int)nw);
    } else {
      e = (a + (it & 7) * 256) % nw;
    }
    if (!on) continue;
    if (OP == 0)
      __hip_atomic_fetch_add(sf + e, 1.0f, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    else if (OP == 1)
      __hip_atomic_fetch_add(su + e, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    else
      __hip_atomic_fetch_add(s64 + e, 3ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
  }
  __syncthreads();
  if (tid == 0) out[blockIdx.x] = (float)s[0];
}

template <int OP, int PAT>
void run(const char* name, float* d, int blocks, int iters) {
  hipEvent_t a, b;
  (void)hipEventCreate(&a);
  (void)hipEventCreate(&b);
  k_lds<OP, PAT><<<blocks, 256>>>(d, iters);        // warm-up
  (void)hipEventRecord(a);
  k_lds<OP, PAT><<<blocks, 256>>>(d, iters);
  (void)hipEventRecord(b);
  (void)hipEventSynchronize(b);
  float ms = 0.f;
  (void)hipEventElapsedTime(&ms, a, b);
  const double active = (PAT == 3 || PAT == 5) ? 0.5 : PAT == 6 ? 0.25 : 1.0;
  const double ops = (double)blocks * 256 * iters * active;
  const double winst = (double)blocks * 4 * iters;   // wave instructions
  std::printf("%-12s pattern %d  %8.3f ms  %9.1f G lane-ops/s  %6.2f lanes/clk/CU  "
              "%6.2f clk/wave-inst/CU\n", name, PAT, ms, ops / ms / 1e6,
              ops / (ms * 1e-3) / 256 / 2.4e9, (ms * 1e-3) * 2.4e9 * 256 / winst);
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
}

int main() {
  float* d = nullptr;
  if (hipMalloc(&d, 65536 * sizeof(float)) != hipSuccess) return 1;
  const int B = 2048, I = 4096;
  run<0, 0>("ds_add_f32", d, B, I);
  run<0, 1>("ds_add_f32", d, B, I);
  run<0, 2>("ds_add_f32", d, B, I);
  run<0, 3>("ds_add_f32", d, B, I);
  run<0, 4>("ds_add_f32", d, B, I);
  run<1, 0>("ds_add_u32", d, B, I);
  run<1, 1>("ds_add_u32", d, B, I);
  run<1, 2>("ds_add_u32", d, B, I);
  run<1, 3>("ds_add_u32", d, B, I);
  run<1, 4>("ds_add_u32", d, B, I);
  run<2, 0>("ds_add_u64", d, B, I);
  run<2, 1>("ds_add_u64", d, B, I);
  run<2, 2>("ds_add_u64", d, B, I);
  run<2, 3>("ds_add_u64", d, B, I);
  run<2, 4>("ds_add_u64", d, B, I);
  run<2, 5>("ds_add_u64", d, B, I);
  run<2, 6>("ds_add_u64", d, B, I);
  run<2, 7>("ds_add_u64", d, B, I);
  run<1, 5>("ds_add_u32", d, B, I);
  run<1, 6>("ds_add_u32", d, B, I);
  (void)hipFree(d);
  return hipDeviceSynchronize() == hipSuccess ? 0 : 1;
}
