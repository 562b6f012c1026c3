// Measured ceilings of the modular products every kernel is built from.
//
// Each thread carries eight independent chains of one product kind in
// registers, long enough that the rate is set by VALU issue alone (no memory
// traffic, and the dependency latency hidden by the eight chains and the
// waves of the other work-groups).  The products are the library's own
// inline functions, so the instruction mix is the one the kernels issue:
//   kind 0  lazy signed FP64 product a w - k q (moduli below 2^46),
//   kind 1  Shoup product by a constant with its companion (60-bit moduli),
//   kind 2  Barrett product of two variable residues (60-bit moduli),
//   kind 3  lazy FP64 butterfly: U + V, U - V with V = a w - k q (one product).
#include "runtime.h"

namespace {

constexpr int CHAINS = 8;

template <int KIND>
__global__ void __launch_bounds__(256) k_modmul_peak(u64* out, u64 iters, u64 q, u64 w, u64 wp, double qf,
                                                     double qinv, double wf, ModConst m) {
  const u64 t = (u64)blockIdx.x * blockDim.x + threadIdx.x;
  u64 acc = 0;
  if (KIND == 0 || KIND == 3) {
    double a[CHAINS], b[CHAINS];
#pragma unroll
    for (int k = 0; k < CHAINS; k++) {
      a[k] = (double)((t * CHAINS + k) % 1000003) - 500001.0;
      b[k] = (double)k;
    }
    for (u64 i = 0; i < iters; i++) {
#pragma unroll
      for (int k = 0; k < CHAINS; k++) {
        if (KIND == 0) {
          a[k] = f64_mulmod_signed(a[k], wf, qf, qinv);
        } else {
          // a butterfly whose output feeds the next one's product: the pair
          // stays bounded by q (U - V and U + V centred again every step)
          const double v = f64_mulmod_signed(a[k], wf, qf, qinv);
          const double u = b[k];
          a[k] = f64_centre(u + v, qf, qinv);
          b[k] = u - v;
          b[k] = b[k] - qf * __builtin_rint(b[k] * qinv);
        }
      }
    }
#pragma unroll
    for (int k = 0; k < CHAINS; k++) acc ^= (u64)__double_as_longlong(a[k] + b[k]);
  } else {
    u64 a[CHAINS];
#pragma unroll
    for (int k = 0; k < CHAINS; k++) a[k] = (t * CHAINS + k) % q;
    for (u64 i = 0; i < iters; i++) {
#pragma unroll
      for (int k = 0; k < CHAINS; k++) {
        if (KIND == 1) a[k] = shoup_mul(a[k], w, wp, q);
        else a[k] = mul_mod(a[k], w + (u64)k, m);
      }
    }
#pragma unroll
    for (int k = 0; k < CHAINS; k++) acc ^= a[k];
  }
  out[t] = acc;
}

}  // namespace

// Rate of `kind` products on the current device: `blocks` x 256 threads, each
// running `iters` steps of eight chains; *rate = products per second.
void modmul_peak(int kind, u64 iters, int blocks, double* rate, double* ms_out) {
  if (kind < 0 || kind > 3) fail(HE_EINVAL, "unknown product kind");
  if (iters < 1 || blocks < 1) fail(HE_EINVAL, "iterations and blocks must be positive");
  // a 40-bit odd modulus for the FP64 kinds, a 60-bit one for the integer kinds (the
  // instruction count does not depend on the modulus being prime)
  const u64 q40 = 1099510054913ull, q60 = 1152921504606584833ull;
  const u64 q = kind == 0 || kind == 3 ? q40 : q60;
  const u64 w = q / 3 + 12345, wp = (u64)(((unsigned __int128)w << 64) / q);
  ModConst m{};
  m.q = q;
  m.bits = 64 - __builtin_clzll(q);
  m.mu = (u64)(((unsigned __int128)1 << (2 * m.bits)) / q);
  const double qf = (double)q, qinv = 1.0 / qf, wf = (double)(w % q40);
  const size_t threads = (size_t)blocks * 256;
  u64* out = nullptr;
  hip_check(hipMalloc(&out, threads * 8), "microbenchmark buffer");
  hipStream_t s = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  auto cleanup = [&] {
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (s) (void)hipStreamDestroy(s);
    (void)hipFree(out);
  };
  try {
    hip_check(hipStreamCreateWithFlags(&s, hipStreamNonBlocking), "stream");
    hip_check(hipEventCreate(&e0), "event");
    hip_check(hipEventCreate(&e1), "event");
    auto launch = [&](u64 it) {
      switch (kind) {
        case 0: hipLaunchKernelGGL(k_modmul_peak<0>, dim3(blocks), dim3(256), 0, s, out, it, q, w, wp, qf, qinv, wf, m); break;
        case 1: hipLaunchKernelGGL(k_modmul_peak<1>, dim3(blocks), dim3(256), 0, s, out, it, q, w, wp, qf, qinv, wf, m); break;
        case 2: hipLaunchKernelGGL(k_modmul_peak<2>, dim3(blocks), dim3(256), 0, s, out, it, q, w, wp, qf, qinv, wf, m); break;
        default: hipLaunchKernelGGL(k_modmul_peak<3>, dim3(blocks), dim3(256), 0, s, out, it, q, w, wp, qf, qinv, wf, m); break;
      }
    };
    launch(iters / 8 + 1);  // warm-up (clocks, code object)
    hip_check(hipEventRecord(e0, s), "event");
    launch(iters);
    hip_check(hipEventRecord(e1, s), "event");
    hip_check(hipEventSynchronize(e1), "microbenchmark");
    float ms = 0;
    hip_check(hipEventElapsedTime(&ms, e0, e1), "event time");
    *rate = (double)threads * (double)iters * CHAINS / (ms * 1e-3);
    if (ms_out) *ms_out = ms;
  } catch (...) {
    cleanup();
    throw;
  }
  cleanup();
}
