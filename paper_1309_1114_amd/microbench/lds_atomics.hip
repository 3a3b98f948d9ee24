// lds_atomics.hip -- LDS atomic-add throughput of one gfx950 chip.
//
// Every workgroup (256 threads) keeps a 16 KiB LDS array; each lane adds to
// an address chosen by the access pattern, `iters` times, with the base
// offset rotating over 8 slots so that consecutive adds do not hit the same
// address.  Printed: lane-operations per second and per clock per CU (256
// CUs, 2.4 GHz), the figures behind the splat's LDS-atomic roofline.
//
//   hipcc --offload-arch=gfx950 -O3 -Xclang -target-feature -Xclang -packed-fp32-ops \
//         -o lds_atomics lds_atomics.hip && ./lds_atomics
#include <hip/hip_runtime.h>

#include <cstdio>

constexpr int kWords = 4096;          // 32-bit words of the LDS array

// op 0: float add, 1: 32-bit integer add, 2: 64-bit integer add
// pattern 0: one address per lane; 1: two lanes per address;
//         2: 64-bit adds at a 24-byte stride (three interleaved channels)
template <int OP, int PAT>
__global__ __launch_bounds__(256) void k_lds(float* out, int iters) {
  __shared__ unsigned int s[kWords];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  for (int i = tid; i < kWords; i += 256) s[i] = 0u;
  __syncthreads();
  const int n64 = kWords / 2;
  unsigned long long* s64 = reinterpret_cast<unsigned long long*>(s);
  int a;
  if (PAT == 0) a = wave * 64 + lane;
  else if (PAT == 1) a = wave * 64 + lane / 2;
  else a = wave * 192 + 3 * lane;
  for (int it = 0; it < iters; ++it) {
    const int slot = (it & 7) * 256;
    if (OP == 0) atomicAdd(reinterpret_cast<float*>(s) + ((a + slot) % kWords), 1.0f);
    else if (OP == 1) atomicAdd(s + ((a + slot) % kWords), 1u);
    else atomicAdd(s64 + ((a + slot) % n64), 3ull);
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
  const double ops = (double)blocks * 256 * iters;
  std::printf("%-12s pattern %d  %8.3f ms  %9.1f G lane-ops/s  %6.2f lanes/clk/CU\n", name, PAT,
              ms, ops / ms / 1e6, ops / (ms * 1e-3) / 256 / 2.4e9);
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
}

int main() {
  float* d = nullptr;
  if (hipMalloc(&d, 65536 * sizeof(float)) != hipSuccess) return 1;
  const int B = 2048, I = 4096;
  run<0, 0>("ds_add_f32", d, B, I / 8);
  run<0, 1>("ds_add_f32", d, B, I / 8);
  run<1, 0>("ds_add_u32", d, B, I);
  run<1, 1>("ds_add_u32", d, B, I);
  run<2, 0>("ds_add_u64", d, B, I);
  run<2, 1>("ds_add_u64", d, B, I);
  run<2, 2>("ds_add_u64", d, B, I);
  (void)hipFree(d);
  return hipDeviceSynchronize() == hipSuccess ? 0 : 1;
}
