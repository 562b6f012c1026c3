// Internal declarations of the MI355X RNS-CKKS library (not part of the ABI).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstring>
#include <map>
#include <memory>
#include <string>
#include <vector>

typedef uint64_t u64;
typedef int64_t i64;
typedef uint32_t u32;
typedef uint16_t u16;
typedef uint8_t u8;

#define HE_MAXMOD 64

// ---------------------------------------------------------------------------
// Per-modulus constants (device resident, one entry per Q or P prime)
// ---------------------------------------------------------------------------
struct ModConst {
  u64 q;
  u64 mu;      // Barrett: floor(2^(2b) / q)
  u32 bits;    // b = bit length of q
  u32 pad;
  u64 ninv;    // N^{-1} mod q
  u64 ninv_sh; // Shoup companion floor(ninv * 2^64 / q)
  u64 r64;     // 2^64 mod q
  u64 r64_sh;
  u64 r96;     // 2^96 mod q
  double qf;   // q and 1/q as doubles (FP64 path, q < 2^50)
  double qinvf;
};

// ---------------------------------------------------------------------------
// Device modular arithmetic (64-bit residues, q < 2^61)
// ---------------------------------------------------------------------------
__device__ __forceinline__ u64 mulhi64(u64 a, u64 b) { return __umul64hi(a, b); }

// a*w mod q for a constant w with companion wp = floor(w 2^64 / q); any a < 2^64.
__device__ __forceinline__ u64 shoup_mul(u64 a, u64 w, u64 wp, u64 q) {
  u64 qh = mulhi64(a, wp);
  u64 r = a * w - qh * q;
  return r >= q ? r - q : r;
}
// a*w mod q for a constant w < q (Shoup companion wp), arithmetic by the size of q
__device__ __forceinline__ u64 mul_const_any(u64 a, u64 w, u64 wp, const ModConst& m);
// lazy variant: result in [0, 2q)
__device__ __forceinline__ u64 shoup_mul_lazy(u64 a, u64 w, u64 wp, u64 q) {
  u64 qh = mulhi64(a, wp);
  return a * w - qh * q;
}

// Barrett reduction of x = hi*2^64 + lo < 2^(2b) (b = bit length of q).
__device__ __forceinline__ u64 barrett_reduce128(u64 hi, u64 lo, const ModConst& m) {
  const u32 b = m.bits;
  u64 t = (lo >> (b - 1)) | (hi << (65 - b));
  u64 th = mulhi64(t, m.mu), tl = t * m.mu;
  u64 qhat = (tl >> (b + 1)) | (th << (63 - b));
  u64 r = lo - qhat * m.q;
  if (r >= m.q) r -= m.q;
  if (r >= m.q) r -= m.q;
  return r;
}
// a*b mod q for a, b < q
__device__ __forceinline__ u64 mul_mod(u64 a, u64 b, const ModConst& m) {
  return barrett_reduce128(mulhi64(a, b), a * b, m);
}

// Exact a*w mod q in FP64 for q < 2^50 and a, w < q: h = a w rounded,
// l = fma(a, w, -h) its exact error, k = rint(h / q); then
// r = fma(-k, q, h) + l = a w - k q exactly (|a w / q - k| < 0.81 keeps the
// fma result below 2^51) and one conditional + q lands it in [0, q).
// Full-rate double operations instead of the quarter-rate 32-bit multipliers.
#define F64_MAX_BITS 50
__device__ __forceinline__ double f64_mulmod(double a, double w, double q, double qinv) {
  const double h = a * w;
  const double l = __fma_rn(a, w, -h);
  const double k = __builtin_rint(h * qinv);
  const double r = __fma_rn(-k, q, h) + l;
  return r < 0.0 ? r + q : r;
}

// Exact conversions between u64 and double for integers in [0, 2^52): the
// value is ORed into the mantissa of 2^52 and 2^52 subtracted (and the
// reverse).  One 32-bit logic op and one double add each way, where the
// general conversions take four to six instructions.
__device__ __forceinline__ double u2d(u64 x) {
  return __longlong_as_double((long long)(x | 0x4330000000000000ull)) - 0x1p52;
}
__device__ __forceinline__ u64 d2u(double x) {
  return (u64)__double_as_longlong(x + 0x1p52) & 0x000FFFFFFFFFFFFFull;
}

// Lazy FP64 arithmetic for q < 2^46: signed representatives are carried
// through sums and butterflies and brought to [0, q) once.
//  * f64_mulmod_signed(a, w), |a| <= 16 q and 0 <= w < q, returns a w - k q
//    exactly with |result| < q: the product's rounding error l satisfies
//    |l| / q < 16 q 2^-53 <= 2^-3, the quotient h * qinv misses h / q by at
//    most 16 q 2^-52 <= 2^-2, so |a w / q - k| < 7/8; h - k q and the final
//    sum are integers below 2^53, hence exact.
//  * sums of up to 64 such terms stay below 2^52 and are exact;
//  * f64_canon(s) for |s| < 2^52 returns s mod q in [0, q); f64_centre(s)
//    a representative of absolute value at most q / 2 + 1.
#define F64_LAZY_BITS 46
__device__ __forceinline__ double f64_mulmod_signed(double a, double w, double q, double qinv) {
  const double h = a * w;
  const double l = __fma_rn(a, w, -h);
  const double k = __builtin_rint(h * qinv);
  return __fma_rn(-k, q, h) + l;
}
__device__ __forceinline__ double f64_centre(double s, double q, double qinv) {
  return __fma_rn(-__builtin_rint(s * qinv), q, s);
}
__device__ __forceinline__ double f64_canon(double s, double q, double qinv) {
  const double r = f64_centre(s, q, qinv);
  return r < 0.0 ? r + q : r;
}

__device__ __forceinline__ u64 mul_const_any(u64 a, u64 w, u64 wp, const ModConst& m) {
  if (m.bits <= F64_MAX_BITS) return d2u(f64_mulmod(u2d(a), u2d(w), m.qf, m.qinvf));
  return shoup_mul(a, w, wp, m.q);
}
// a*b mod q, choosing the arithmetic by the size of q (same residue either way)
__device__ __forceinline__ u64 mul_mod_any(u64 a, u64 b, const ModConst& m) {
  if (m.bits <= F64_MAX_BITS) return d2u(f64_mulmod(u2d(a), u2d(b), m.qf, m.qinvf));
  return mul_mod(a, b, m);
}
__device__ __forceinline__ u64 add_mod(u64 a, u64 b, u64 q) {
  u64 s = a + b;
  return s >= q ? s - q : s;
}
__device__ __forceinline__ u64 sub_mod(u64 a, u64 b, u64 q) { return a >= b ? a - b : a + q - b; }
// any 64-bit value mod q
__device__ __forceinline__ u64 reduce64(u64 x, const ModConst& m) { return barrett_reduce128(0, x, m); }
// signed 64-bit value mod q
__device__ __forceinline__ u64 reduce_signed(i64 v, const ModConst& m) {
  if (v >= 0) return reduce64((u64)v, m);
  u64 r = reduce64((u64)(-v), m);
  return r ? m.q - r : 0;
}

// ---------------------------------------------------------------------------
// Host-side objects
// ---------------------------------------------------------------------------
// Stream-ordered caching pool over hipMalloc.  All work of a context runs on
// its stream, so a block released here may be handed to a later launch on
// the same stream immediately.
struct DevPool {
  std::multimap<size_t, void*> free_;
  std::map<void*, size_t> live_;
  size_t bytes_live = 0, bytes_cached = 0, peak = 0;
  void* (*user_alloc)(size_t, void*) = nullptr;
  void (*user_release)(void*, void*) = nullptr;
  void* user = nullptr;
  // the stream every block of this pool was last used on (the owning
  // context's): trim waits for it alone, so trimming one context does not
  // stall the others
  hipStream_t stream = nullptr;
  // while set, allocations come from (and blocks of it return to) this pool:
  // the private arena of a HIP graph being recorded
  DevPool* redirect = nullptr;
  // a frozen pool serves only cached blocks (no device allocation, which a
  // stream capture must not see)
  bool frozen = false;
  // serve only cached blocks of exactly the requested size (an arena sized by
  // one run serves a repeat of the same run)
  bool exact = false;
  // a fixed device region handed out front to back, never given back (the
  // workspace of the allocation-free entry points; reset by the caller)
  char* bump_base = nullptr;
  size_t bump_cap = 0, bump_off = 0;
  void* get(size_t bytes);
  void put(void* p);
  void trim();
  void wait();
  ~DevPool();
};

struct DevBuf {
  DevPool* pool = nullptr;
  u64* p = nullptr;
  size_t words = 0;
  DevBuf() {}
  DevBuf(DevPool* pl, size_t w) : pool(pl), words(w) { p = (u64*)pl->get(w * 8); }
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  DevBuf(DevBuf&& o) noexcept : pool(o.pool), p(o.p), words(o.words) { o.p = nullptr; }
  DevBuf& operator=(DevBuf&& o) noexcept {
    release();
    pool = o.pool; p = o.p; words = o.words; o.p = nullptr;
    return *this;
  }
  void release() { if (p && pool) pool->put(p); p = nullptr; }
  ~DevBuf() { release(); }
};

// B ciphertexts at one level and scale (or elements of R_{Q_l P}^2 when qp =
// true), stacked as u64[2][B][nlimbs][N]: poly(p) holds component p of every
// member contiguously, so a batch is just more limbs for every kernel.
struct HeCt {
  u64 N = 0;
  int level = 0;
  bool qp = false;
  // limbs of FP64 moduli stored packed (a product side's ModDown output,
  // read only by the tensor sums; every other operation takes unpacked
  // elements)
  bool packed = false;
  int nlimbs = 0;
  int B = 1;
  double scale = 1.0;
  DevBuf d;
  u64* poly(int p) const { return d.p + (size_t)p * B * nlimbs * N; }
  u64* limb(int p, int k) const { return d.p + ((size_t)p * B * nlimbs + k) * N; }
  // member b, component p
  u64* member(int p, int b) const { return d.p + ((size_t)p * B + b) * nlimbs * N; }
  size_t polys() const { return (size_t)2 * B; }
};
