// gfx950 kernels of the RNS-CKKS matrix-product path.
//
// Residues are 64-bit words in [0, q) with q < 2^61, limb-major
// (u64[limbs][N]).  Products by constants use Shoup's method (precomputed
// floor(w 2^64 / q)); products of two variables use Barrett reduction of the
// 128-bit product.  Every kernel computes an exactly defined integer result,
// so fusion and reordering never change a residue.
#include "kernels.h"

#include <cstdio>
#include <type_traits>

#define TPB 256
#define NTT_LDS 4096  // u64 words of LDS per NTT work-group (32 KiB)

static inline int cdiv(u64 a, u64 b) { return (int)((a + b - 1) / b); }

// Launch-shape knobs (process-wide).  They change how work is grouped into
// launches, never a residue; the autotuner picks them by timing.
namespace {
struct Knobs {
  int ms_members = 8;   // batch members per key-inner-product launch (1..8)
  int mr_members = 8;   // batch members per multi-rotation launch (1..8)
  int mr_rotations = 64;  // rotations per multi-rotation launch (1..64)
  int ntt_interleave = 0;  // block passes visit limbs of one modulus back to back (0/1)
  int ew_interleave = 1;   // plaintext-broadcast sums visit the limbs sharing a plaintext back to back (0/1)
  int cov_row_blocks = 4;  // row blocks of a covariance stacked into one batch (1..8)
  int mr_int_split = 1;    // 60-bit limbs of a multi-rotation launch in their own kernel (0/1)
  int mr_int_pass = 4;     // members per pass of that kernel (4/8)
  int mr_int_chunk = 64;   // rotations per dispatch chunk of that kernel (1..64)
  int mr_int_concurrent = 0;  // that kernel on a forked stream, beside the FP64 one (0/1)
  int mr_group = 4;        // rotations per work-group of a multi-rotation launch, sharing the digit loads (1/2/4)
  int fbc_mfma = 1;        // ModDown's lift as an int8 matrix product (0/1)
  int xcd_map = 1;         // the MFMA lift's work-groups of one polynomial kept on one XCD (0/1)
  int sum_streams = 4;     // term streams sharing a plaintext per thread of the multi-output sums (1/2/4)
  int mr_pair = 1;         // the A side's two masked multi-rotation launches as one (0/1)
  // stage split of the register-blocked NTT per ring size (index log N):
  // 0 = the default, 1 = one stage moved between the column and block passes
  int ntt_split[17] = {};
} g_knobs;
}
bool knob_set(const char* name, int v) {
  std::string n(name);
  if (n == "ms_members" && v >= 1 && v <= 8) g_knobs.ms_members = v;
  else if (n == "mr_members" && v >= 1 && v <= 8) g_knobs.mr_members = v;
  else if (n == "mr_rotations" && v >= 1 && v <= MR_MAX) g_knobs.mr_rotations = v;
  else if (n == "ntt_interleave" && (v == 0 || v == 1)) g_knobs.ntt_interleave = v;
  else if (n == "ew_interleave" && (v == 0 || v == 1)) g_knobs.ew_interleave = v;
  else if (n == "cov_row_blocks" && v >= 1 && v <= 8) g_knobs.cov_row_blocks = v;
  else if (n == "mr_group" && (v == 1 || v == 2 || v == 4)) g_knobs.mr_group = v;
  else if (n == "mr_int_split" && (v == 0 || v == 1)) g_knobs.mr_int_split = v;
  else if (n == "mr_int_pass" && (v == 4 || v == 8)) g_knobs.mr_int_pass = v;
  else if (n == "mr_int_chunk" && v >= 1 && v <= MR_MAX) g_knobs.mr_int_chunk = v;
  else if (n == "mr_int_concurrent" && (v == 0 || v == 1)) g_knobs.mr_int_concurrent = v;
  else if (n == "fbc_mfma" && (v == 0 || v == 1)) g_knobs.fbc_mfma = v;
  else if (n == "xcd_map" && (v == 0 || v == 1)) g_knobs.xcd_map = v;
  else if (n == "sum_streams" && (v == 1 || v == 2 || v == 4)) g_knobs.sum_streams = v;
  else if (n == "mr_pair" && (v == 0 || v == 1)) g_knobs.mr_pair = v;
  else if ((n == "ntt_split_13" || n == "ntt_split_14" || n == "ntt_split_15") && (v == 0 || v == 1))
    g_knobs.ntt_split[std::stoi(n.substr(10))] = v;
  else return false;
  return true;
}
bool knob_get(const char* name, int* v) {
  std::string n(name);
  if (n == "ms_members") *v = g_knobs.ms_members;
  else if (n == "mr_members") *v = g_knobs.mr_members;
  else if (n == "mr_rotations") *v = g_knobs.mr_rotations;
  else if (n == "ntt_interleave") *v = g_knobs.ntt_interleave;
  else if (n == "ew_interleave") *v = g_knobs.ew_interleave;
  else if (n == "cov_row_blocks") *v = g_knobs.cov_row_blocks;
  else if (n == "mr_group") *v = g_knobs.mr_group;
  else if (n == "mr_int_split") *v = g_knobs.mr_int_split;
  else if (n == "mr_int_pass") *v = g_knobs.mr_int_pass;
  else if (n == "mr_int_chunk") *v = g_knobs.mr_int_chunk;
  else if (n == "mr_int_concurrent") *v = g_knobs.mr_int_concurrent;
  else if (n == "fbc_mfma") *v = g_knobs.fbc_mfma;
  else if (n == "xcd_map") *v = g_knobs.xcd_map;
  else if (n == "sum_streams") *v = g_knobs.sum_streams;
  else if (n == "mr_pair") *v = g_knobs.mr_pair;
  else if (n == "ntt_split_13" || n == "ntt_split_14" || n == "ntt_split_15") *v = g_knobs.ntt_split[std::stoi(n.substr(10))];
  else return false;
  return true;
}

// Stage splits (GA + GB stages in the column pass, GC + GD in the block pass,
// each group at most 4: sixteen values per thread) of the register-blocked
// NTT.  The tile is 4096 words: the column pass needs GA + GB <= 8 (R <= 256
// rows in LDS) and the block pass GC + GD >= 6 (at most 64 blocks).  Split 1
// (knob ntt_split_<log N>) moves one stage from one pass to the other.
template <int LOGN_, int GA_, int GB_, int GC_, int GD_>
struct NttSplit {
  static constexpr int LOGN = LOGN_, GA = GA_, GB = GB_, GC = GC_, GD = GD_;
  static_assert(GA + GB + GC + GD == LOGN && GA + GB <= 8 && GC + GD >= 6, "stage split");
  static_assert(GA >= 1 && GA <= 4 && GB >= 1 && GB <= 4 && GC >= 1 && GC <= 4 && GD >= 1 && GD <= 4, "groups");
};
template <class F>
static bool ntt_dispatch(int logN, F&& f) {
  const int alt = logN >= 13 && logN <= 15 ? g_knobs.ntt_split[logN] : 0;
  switch (logN * 2 + alt) {
    case 32: f(NttSplit<16, 4, 4, 4, 4>{}); return true;
    case 30: f(NttSplit<15, 4, 3, 4, 4>{}); return true;
    case 31: f(NttSplit<15, 4, 4, 4, 3>{}); return true;
    case 28: f(NttSplit<14, 4, 3, 4, 3>{}); return true;
    case 29: f(NttSplit<14, 4, 4, 3, 3>{}); return true;
    case 26: f(NttSplit<13, 3, 3, 4, 3>{}); return true;
    case 27: f(NttSplit<13, 4, 3, 3, 3>{}); return true;
    case 24: f(NttSplit<12, 3, 3, 3, 3>{}); return true;
    default: return false;
  }
}
#define NTT_SPLIT_ARGS S::LOGN, S::GA, S::GB, S::GC, S::GD

// ---------------------------------------------------------------------------
// Optional per-family device timing: HIP events recorded on the launching
// stream around each launch while enabled.
// ---------------------------------------------------------------------------
// Algorithmic modular products of a launch by arithmetic: moduli below 2^46
// take the lazy FP64 product, the others 64-bit integer products.
Mm mm_map(const DeviceTables& T, const LimbMap& m, int nlimbs, double per_limb) {
  Mm r;
  for (int k = 0; k < nlimbs; k++) {
    const int idx = m.idx[k % m.n];
    if (idx >= 0) r.add(T.bits[idx], per_limb);
  }
  return r;
}
// limbs of q_0 .. q_{nq-1}, `reps` times
static Mm mm_q(const DeviceTables& T, int nq, double per_limb, double reps = 1.0) {
  Mm r;
  for (int k = 0; k < nq; k++) r.add(T.bits[k], per_limb * reps);
  return r;
}
// an R_{Q_l P} element's positions: q_0 .. q_{nq-1}, then the special primes
static Mm mm_qp(const DeviceTables& T, int nq, int nqp, int L, double per_q, double per_p, double reps = 1.0) {
  Mm r;
  for (int pos = 0; pos < nqp; pos++) {
    const int m = pos < nq ? pos : L + 1 + (pos - nq);
    r.add(T.bits[m], (pos < nq ? per_q : per_p) * reps);
  }
  return r;
}
static Mm operator+(Mm a, const Mm& b) {
  a.f += b.f;
  a.i += b.i;
  return a;
}

namespace {
struct ProfPair {
  hipEvent_t a, b;
};
bool g_prof_on = false;
std::map<std::string, std::vector<ProfPair>> g_prof;
struct ProfTotal {
  double ms = 0, bytes = 0, mm_f64 = 0, mm_int = 0, unit_bytes = 0;
  u64 launches = 0;
};
std::map<std::string, ProfTotal> g_prof_done;
std::map<std::string, double> g_prof_bytes;
std::map<std::string, Mm> g_prof_mm;
std::map<std::string, double> g_prof_unit;
std::vector<hipEvent_t> g_ev_free;
hipEvent_t ev_get() {
  if (!g_ev_free.empty()) {
    hipEvent_t e = g_ev_free.back();
    g_ev_free.pop_back();
    return e;
  }
  hipEvent_t e;
  (void)hipEventCreate(&e);
  return e;
}
// `bytes` = algorithmic HBM bytes of the launch (every input read once,
// every output written once); `mm` = its algorithmic modular products (NTT
// butterflies, basis-conversion and inner-product terms), by arithmetic
struct ProfScope {
  const char* name;
  hipStream_t s;
  hipEvent_t a = nullptr;
  // `unit` = the bytes of the launch's work counted in the rotation's unit
  // (each key read once per launch, each member's ciphertext in and out once
  // per rotation); the kernel-I/O bytes when not given
  ProfScope(const char* n, hipStream_t st, double bytes = 0, Mm mm = Mm(), double unit = -1.0) : name(n), s(st) {
    if (g_prof_on) {
      a = ev_get();
      (void)hipEventRecord(a, s);
      g_prof_bytes[name] += bytes;
      g_prof_unit[name] += unit >= 0 ? unit : bytes;
      g_prof_mm[name].f += mm.f;
      g_prof_mm[name].i += mm.i;
    }
  }
  ~ProfScope() {
    if (a) {
      hipEvent_t b = ev_get();
      (void)hipEventRecord(b, s);
      g_prof[name].push_back({a, b});
    }
  }
};
void prof_collect() {
  for (auto& kv : g_prof) {
    auto& acc = g_prof_done[kv.first];
    for (auto& p : kv.second) {
      float ms = 0;
      (void)hipEventSynchronize(p.b);
      (void)hipEventElapsedTime(&ms, p.a, p.b);
      acc.ms += ms;
      acc.launches += 1;
      g_ev_free.push_back(p.a);
      g_ev_free.push_back(p.b);
    }
    kv.second.clear();
  }
  for (auto& kv : g_prof_bytes) g_prof_done[kv.first].bytes += kv.second;
  g_prof_bytes.clear();
  for (auto& kv : g_prof_mm) {
    g_prof_done[kv.first].mm_f64 += kv.second.f;
    g_prof_done[kv.first].mm_int += kv.second.i;
  }
  g_prof_mm.clear();
  for (auto& kv : g_prof_unit) g_prof_done[kv.first].unit_bytes += kv.second;
  g_prof_unit.clear();
}
}  // namespace

hipError_t copy_async(const char* family, void* dst, const void* src, size_t bytes, hipStream_t s) {
  ProfScope ps(family, s, 2.0 * (double)bytes);
  return hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToDevice, s);
}
hipError_t copy2d_async(const char* family, void* dst, size_t dpitch, const void* src, size_t spitch, size_t width,
                        size_t height, hipStream_t s) {
  ProfScope ps(family, s, 2.0 * (double)width * (double)height);
  return hipMemcpy2DAsync(dst, dpitch, src, spitch, width, height, hipMemcpyDeviceToDevice, s);
}

bool prof_enabled() { return g_prof_on; }
void prof_enable(bool on) {
  prof_collect();
  if (on) g_prof_done.clear();
  g_prof_on = on;
}
bool prof_read(const char* family, double* ms, u64* launches, double* bytes) {
  prof_collect();
  auto it = g_prof_done.find(family);
  if (it == g_prof_done.end()) {
    *ms = 0;
    *launches = 0;
    *bytes = 0;
    return false;
  }
  *ms = it->second.ms;
  *launches = it->second.launches;
  *bytes = it->second.bytes;
  return true;
}
bool prof_read_ops(const char* family, double* mm_f64, double* mm_int, double* unit_bytes) {
  prof_collect();
  auto it = g_prof_done.find(family);
  *mm_f64 = it == g_prof_done.end() ? 0 : it->second.mm_f64;
  *mm_int = it == g_prof_done.end() ? 0 : it->second.mm_int;
  *unit_bytes = it == g_prof_done.end() ? 0 : it->second.unit_bytes;
  return it != g_prof_done.end();
}
std::vector<std::string> prof_families() {
  prof_collect();
  std::vector<std::string> r;
  for (auto& kv : g_prof_done) r.push_back(kv.first);
  return r;
}

__device__ __forceinline__ int limb_mod(const LimbMap& m, int k) { return m.idx[k % m.n]; }
__device__ __forceinline__ size_t limb_slot(const LimbMap& m, int k) {
  return m.slot_per > 0 ? (size_t)(k / m.slot_per) * m.slot_stride + m.slot_off + k % m.slot_per : (size_t)k;
}
// Limb of grid row y when `outer` groups of gridDim.y / outer limbs are
// visited interleaved (limb j of every group, then limb j + 1, ...): limbs
// that share a modulus or a broadcast operand then run back to back, and
// when a row's work-groups always land on the same XCDs (row length a
// multiple of 8), the shared data is served from L2.  outer <= 1: y itself.
__device__ __forceinline__ int grid_limb(int y, int outer) {
  if (outer <= 1) return y;
  const int inner = gridDim.y / outer;
  return (y % outer) * inner + y / outer;
}
// Work-group -> (coefficient block, limb) for the multiply-sums whose limbs
// come in `outer` groups of `inner` limbs, limb g * inner + t using broadcast
// operand t: with a 1-D grid, the `outer` limbs that share operand t at one
// coefficient block get consecutive ids of one residue mod 8, so they run back
// to back on one XCD and the shared block comes from its L2.  outer <= 1:
// the 2-D grid (x = block, y = limb).
__device__ __forceinline__ void block_limb(int outer, int inner, int nblk, int& blk, int& k) {
  if (outer <= 1) {
    blk = blockIdx.x;
    k = blockIdx.y;
    return;
  }
  const int id = blockIdx.x;
  const int xcd = id & 7;
  int r = id >> 3;
  const int g = r % outer;
  r /= outer;
  const int nhi = nblk >> 3;
  blk = (r % nhi) * 8 + xcd;
  k = g * inner + r / nhi;
}
// launch shape for block_limb: nl limbs in groups sharing a period of bl
static inline dim3 sum_grid(int nblk, int nl, int bl, int knob, int& outer) {
  outer = (knob && bl > 0 && nl > bl && nl % bl == 0 && nblk % 8 == 0) ? nl / bl : 1;
  return outer > 1 ? dim3((unsigned)(nblk * nl)) : dim3(nblk, nl);
}
// host side: the interleave factor for nlimbs limbs in groups of `period`
static inline int interleave_of(int nlimbs, int period, int knob) {
  return (knob && period > 0 && nlimbs > period && nlimbs % period == 0) ? nlimbs / period : 1;
}
// the shortest period of a limb map's moduli (skipped limbs match anything)
static inline int modulus_period(const LimbMap& m) {
  for (int p = 1; p < m.n; p++) {
    if (m.n % p) continue;
    bool ok = true;
    for (int k = p; k < m.n && ok; k++) {
      const int a = m.idx[k], b = m.idx[k % p];
      ok = a < 0 || b < 0 || a == b;
    }
    if (ok) return p;
  }
  return m.n;
}

__device__ __forceinline__ u32 brv(u32 x, int bits) { return __brev(x) >> (32 - bits); }

// ---------------------------------------------------------------------------
// Negacyclic NTT.  Forward: natural-order coefficients -> evaluations with
// index i holding a(psi^(2 brv(i)+1)) (Cooley-Tukey butterflies, twiddles
// psi^brv).  Inverse: Gentleman-Sande with psi^-brv, then N^{-1}.
//
// The log N stages are split in two LDS passes.  With R = 2^s1 rows and
// T1 = N / R columns: the first s1 stages pair elements of one column
// (stride >= T1), the last s2 = log N - s1 stages pair elements inside one
// contiguous block of T1 words.  Each pass loads a tile into LDS once, runs
// its stages there and writes back once.
// ---------------------------------------------------------------------------
struct NttShape {
  int logN, s1, R, T1, C, K;
};
static NttShape ntt_shape(int logN) {
  NttShape sh;
  sh.logN = logN;
  sh.s1 = logN / 2;
  sh.R = 1 << sh.s1;
  sh.T1 = 1 << (logN - sh.s1);
  sh.C = NTT_LDS / sh.R;
  if (sh.C > sh.T1) sh.C = sh.T1;
  sh.K = NTT_LDS / sh.T1;
  if (sh.K > sh.R) sh.K = sh.R;
  return sh;
}

// Column pass: forward stages [0, s1) / inverse stages [s2, logN).
__global__ void __launch_bounds__(TPB) k_ntt_cols(u64* data, LimbMap map, int logN, int R, int T1, int C,
                                                  int inverse, const u64* __restrict__ tw,
                                                  const u64* __restrict__ twsh, const ModConst* __restrict__ mc) {
  __shared__ u64 sh[NTT_LDS];
  const int limb = blockIdx.y;
  const int m = limb_mod(map, limb);
  if (m < 0) return;
  const u64 N = 1ull << logN;
  u64* a = data + limb_slot(map, limb) * N;
  const int c0 = blockIdx.x * C;
  const int tot = R * C;
  for (int e = threadIdx.x; e < tot; e += TPB) {
    int r = e / C, c = e - r * C;
    sh[e] = a[(size_t)r * T1 + c0 + c];
  }
  __syncthreads();
  const ModConst mk = mc[m];
  const u64 q = mk.q;
  const u64* w = tw + (size_t)m * N;
  const u64* wsh = twsh + (size_t)m * N;
  const int nbf = tot >> 1;
  if (!inverse) {
    int s = 0;
    for (int half = R >> 1; half >= 1; half >>= 1, s++) {
      for (int b = threadIdx.x; b < nbf; b += TPB) {
        int c = b % C, bb = b / C;
        int i = bb / half, rr = bb - i * half;
        int r = 2 * i * half + rr;
        u64 W = w[(1 << s) + i], Wp = wsh[(1 << s) + i];
        u64 U = sh[r * C + c];
        u64 V = shoup_mul(sh[(r + half) * C + c], W, Wp, q);
        sh[r * C + c] = add_mod(U, V, q);
        sh[(r + half) * C + c] = sub_mod(U, V, q);
      }
      __syncthreads();
    }
    for (int e = threadIdx.x; e < tot; e += TPB) {
      int r = e / C, c = e - r * C;
      a[(size_t)r * T1 + c0 + c] = sh[e];
    }
  } else {
    // global GS stages with t = half*T1, h = R / (2 half)
    for (int half = 1; half < R; half <<= 1) {
      int h = R / (2 * half);
      for (int b = threadIdx.x; b < nbf; b += TPB) {
        int c = b % C, bb = b / C;
        int i = bb / half, rr = bb - i * half;
        int r = 2 * i * half + rr;
        u64 W = w[h + i], Wp = wsh[h + i];
        u64 U = sh[r * C + c], V = sh[(r + half) * C + c];
        sh[r * C + c] = add_mod(U, V, q);
        sh[(r + half) * C + c] = shoup_mul(sub_mod(U, V, q), W, Wp, q);
      }
      __syncthreads();
    }
    for (int e = threadIdx.x; e < tot; e += TPB) {
      int r = e / C, c = e - r * C;
      a[(size_t)r * T1 + c0 + c] = shoup_mul(sh[e], mk.ninv, mk.ninv_sh, q);
    }
  }
}

// Block pass: forward stages [s1, logN) / inverse stages [0, s2), on K
// contiguous blocks of T1 words per work-group.
__global__ void __launch_bounds__(TPB) k_ntt_rows(u64* data, LimbMap map, int logN, int s1, int T1, int K,
                                                  int inverse, const u64* __restrict__ tw,
                                                  const u64* __restrict__ twsh, const ModConst* __restrict__ mc) {
  __shared__ u64 sh[NTT_LDS];
  const int limb = blockIdx.y;
  const int m = limb_mod(map, limb);
  if (m < 0) return;
  const u64 N = 1ull << logN;
  const int blk0 = blockIdx.x * K;
  u64* a = data + limb_slot(map, limb) * N + (size_t)blk0 * T1;
  const int tot = K * T1;
  for (int e = threadIdx.x; e < tot; e += TPB) sh[e] = a[e];
  __syncthreads();
  const u64 q = mc[m].q;
  const u64* w = tw + (size_t)m * N;
  const u64* wsh = twsh + (size_t)m * N;
  const int nbf = tot >> 1;
  if (!inverse) {
    int sp = 0;
    for (int t = T1 >> 1; t >= 1; t >>= 1, sp++) {
      for (int b = threadIdx.x; b < nbf; b += TPB) {
        int blk = b / (T1 >> 1), lb = b - blk * (T1 >> 1);
        int i = lb / t, rr = lb - i * t;
        int lo = 2 * i * t + rr;
        int hi = blk0 + blk;
        int widx = (1 << (s1 + sp)) + (hi << sp) + i;
        u64 W = w[widx], Wp = wsh[widx];
        int x = blk * T1 + lo;
        u64 U = sh[x];
        u64 V = shoup_mul(sh[x + t], W, Wp, q);
        sh[x] = add_mod(U, V, q);
        sh[x + t] = sub_mod(U, V, q);
      }
      __syncthreads();
    }
  } else {
    for (int t = 1; t < T1; t <<= 1) {
      for (int b = threadIdx.x; b < nbf; b += TPB) {
        int blk = b / (T1 >> 1), lb = b - blk * (T1 >> 1);
        int i = lb / t, rr = lb - i * t;
        int lo = 2 * i * t + rr;
        int hi = blk0 + blk;
        // global group index j/(2t) = hi*T1/(2t) + i ; h = N/(2t)
        u64 h = N / (2 * (u64)t);
        u64 widx = h + (u64)hi * (T1 / (2 * t)) + i;
        u64 W = w[widx], Wp = wsh[widx];
        int x = blk * T1 + lo;
        u64 U = sh[x], V = sh[x + t];
        sh[x] = add_mod(U, V, q);
        sh[x + t] = shoup_mul(sub_mod(U, V, q), W, Wp, q);
      }
      __syncthreads();
    }
  }
  for (int e = threadIdx.x; e < tot; e += TPB) a[e] = sh[e];
}

// ---------------------------------------------------------------------------
// Register-blocked NTT (log N = 12..16).  Each pass streams a 4096-word tile
// through LDS once; inside the pass every thread holds 2^G residues in
// registers and runs G consecutive butterfly stages on them (G <= 4), twice,
// with one LDS exchange in between.
//
// Forward stage s (Cooley-Tukey) pairs bit logN-1-s of the index with twiddle
// psi^brv at 2^s + (x >> (logN - s)).  A thread's values v[r] sit at
// x = base + (r << (logN - s0 - G)); with hi = base >> (logN - s0) the
// twiddle of stage s0 + j is at 2^(s0+j) + (hi << j) + (r >> (G - j)).
// Inverse stage on bit b (Gentleman-Sande) uses psi^-brv at
// 2^(logN-1-b) + (x >> (b+1)); values at x = base + (r << b0), hi = base >> (b0 + G).
//
// Two arithmetics, chosen per limb (uniform over a work-group):
//  * Shoup: 64-bit words, w * a mod q with the companion floor(w 2^64 / q)
//    (any q < 2^61; the 64-bit products run on the quarter-rate 32-bit
//    multipliers);
//  * lazy FP64 for q < 2^46: values are signed doubles; a butterfly is one
//    exact signed product a w - k q (|.| < q for |a| <= 16 q, see
//    f64_mulmod_signed), one add and one subtract, with no conditional
//    corrections.  Forward (Cooley-Tukey) stages add at most q to the bound,
//    so the eight stages of a pass stay below 9 q; inverse (Gentleman-Sande)
//    stages double it, so each group of four stages starts from a centred
//    value (reduce) and ends below 16 q.  Stores to memory bring values to
//    [0, q).  Every operation is a full-rate double op.
// Both give the same residues.
// ---------------------------------------------------------------------------
struct ShoupArith {
  typedef u64 V;
  const u64* __restrict__ w;
  const u64* __restrict__ wsh;
  u64 q, ninv, ninv_sh;
  __device__ __forceinline__ V load(u64 x) const { return x; }
  __device__ __forceinline__ u64 store(V x) const { return x; }
  __device__ __forceinline__ V reduce(V x) const { return x; }
  __device__ __forceinline__ V add(V a, V b) const { return add_mod(a, b, q); }
  __device__ __forceinline__ V sub(V a, V b) const { return sub_mod(a, b, q); }
  __device__ __forceinline__ V mulw(V a, u32 i) const { return shoup_mul(a, w[i], wsh[i], q); }
  __device__ __forceinline__ V scale_ninv(V a) const { return shoup_mul(a, ninv, ninv_sh, q); }
};

struct F64LazyArith {
  typedef double V;
  const double* __restrict__ w;
  double q, qinv, ninv;
  __device__ __forceinline__ V load(u64 x) const { return u2d(x); }
  __device__ __forceinline__ u64 store(V x) const { return d2u(f64_canon(x, q, qinv)); }
  __device__ __forceinline__ V reduce(V x) const { return f64_centre(x, q, qinv); }
  __device__ __forceinline__ V add(V a, V b) const { return a + b; }
  __device__ __forceinline__ V sub(V a, V b) const { return a - b; }
  __device__ __forceinline__ V mulw(V a, u32 i) const { return f64_mulmod_signed(a, w[i], q, qinv); }
  __device__ __forceinline__ V scale_ninv(V a) const { return f64_mulmod_signed(a, ninv, q, qinv); }
};

template <int G, class A>
__device__ __forceinline__ void fwd_group(typename A::V (&v)[16], int s0, u32 hi, const A& ar) {
#pragma unroll
  for (int j = 0; j < G; j++) {
    const int half = 1 << (G - 1 - j);
#pragma unroll
    for (int r = 0; r < (1 << G); r++) {
      if (r & half) continue;
      const u32 widx = (1u << (s0 + j)) + (hi << j) + (u32)(r >> (G - j));
      const typename A::V U = v[r];
      const typename A::V V = ar.mulw(v[r + half], widx);
      v[r] = ar.add(U, V);
      v[r + half] = ar.sub(U, V);
    }
  }
}

// The forward block pass's last G stages (s0 = log N - G, hi < 2^s0): any
// arithmetic takes the twiddles from the table ...
template <int G, class A>
__device__ __forceinline__ void fwd_group_last(typename A::V (&v)[16], int s0, u32 hi, const A& ar) {
  fwd_group<G>(v, s0, hi, ar);
}
// ... but the lazy FP64 one computes them: with W[k] = psi^brv(k),
//   W[2^(s0+j) + (hi << j) + low] = W[2^(s0+j) + low] * Y^(2^(G-1-j)),
//   Y = W[hi << (G-1)]
// (bit reversal splits over the disjoint bit fields, and brv(hi) has its low
// G bits clear).  One table load and G - 1 squarings per thread, then one
// product per twiddle, against 2^G - 1 distinct table loads per thread: the
// table W[2^(s0+j) + low] has 2^G - 1 entries shared by the whole grid.
template <int G>
__device__ __forceinline__ void fwd_group_last(double (&v)[16], int s0, u32 hi, const F64LazyArith& ar) {
  double P[G];
  P[G - 1] = ar.w[hi << (G - 1)];
#pragma unroll
  for (int j = G - 2; j >= 0; j--) P[j] = f64_mulmod_signed(P[j + 1], P[j + 1], ar.q, ar.qinv);
#pragma unroll
  for (int j = 0; j < G; j++) {
    const int half = 1 << (G - 1 - j);
    double w[1 << (G - 1)];
#pragma unroll
    for (int low = 0; low < (1 << j); low++)
      w[low] = f64_mulmod_signed(ar.w[(1u << (s0 + j)) + low], P[j], ar.q, ar.qinv);
#pragma unroll
    for (int r = 0; r < (1 << G); r++) {
      if (r & half) continue;
      const double U = v[r];
      const double V = f64_mulmod_signed(v[r + half], w[r >> (G - j)], ar.q, ar.qinv);
      v[r] = U + V;
      v[r + half] = U - V;
    }
  }
}

template <int G, class A>
__device__ __forceinline__ void inv_group(typename A::V (&v)[16], int b0, int logN, u32 hi, const A& ar) {
#pragma unroll
  for (int j = 0; j < G; j++) {
    const int half = 1 << j;
#pragma unroll
    for (int r = 0; r < (1 << G); r++) {
      if (r & half) continue;
      const u32 widx = (1u << (logN - 1 - b0 - j)) + (hi << (G - j - 1)) + (u32)(r >> (j + 1));
      const typename A::V U = v[r], V = v[r + half];
      v[r] = ar.add(U, V);
      v[r + half] = ar.mulw(ar.sub(U, V), widx);
    }
  }
}

// The inverse block pass's first G stages (b0 = 0, hi < 2^(log N - G)): the
// twiddle of stage j is W'[2^(log N - 1 - j) + (hi << (G - 1 - j)) + low],
// W'[k] = psi^-brv(k), the index pattern of the forward pass's last stages,
// so the lazy FP64 arithmetic computes them the same way (fwd_group_last):
// one table load and G - 1 squarings per thread, then one product per
// twiddle from the small table W'[2^(log N - 1 - j) + low] shared by the
// grid.  Any other arithmetic reads the table.
template <int G, class A>
__device__ __forceinline__ void inv_group_first(typename A::V (&v)[16], int logN, u32 hi, const A& ar) {
  inv_group<G>(v, 0, logN, hi, ar);
}
template <int G>
__device__ __forceinline__ void inv_group_first(double (&v)[16], int logN, u32 hi, const F64LazyArith& ar) {
  double P[G];
  P[G - 1] = ar.w[hi << (G - 1)];
#pragma unroll
  for (int jj = G - 2; jj >= 0; jj--) P[jj] = f64_mulmod_signed(P[jj + 1], P[jj + 1], ar.q, ar.qinv);
#pragma unroll
  for (int j = 0; j < G; j++) {
    const int half = 1 << j, jj = G - 1 - j;
    double w[1 << (G - 1)];
#pragma unroll
    for (int low = 0; low < (1 << jj); low++)
      w[low] = f64_mulmod_signed(ar.w[(1u << (logN - 1 - j)) + low], P[jj], ar.q, ar.qinv);
#pragma unroll
    for (int r = 0; r < (1 << G); r++) {
      if (r & half) continue;
      const double U = v[r], V = v[r + half];
      v[r] = U + V;
      v[r + half] = f64_mulmod_signed(U - V, w[r >> (j + 1)], ar.q, ar.qinv);
    }
  }
}
// The inverse column pass's last G stages followed by the scaling by N^-1:
// the final stage has the single twiddle W'[1], so its two outputs are
// (U + V) N^-1 and (U - V) (W'[1] N^-1): the lazy FP64 arithmetic folds the
// scaling into that stage (two products per butterfly where the stage and
// the scaling took three).  Any other arithmetic scales afterwards.
template <int G, class A>
__device__ __forceinline__ void inv_group_last_scaled(typename A::V (&v)[16], int b0, int logN, const A& ar) {
  inv_group<G>(v, b0, logN, 0u, ar);
#pragma unroll
  for (int mm = 0; mm < (1 << G); mm++) v[mm] = ar.scale_ninv(v[mm]);
}
template <int G>
__device__ __forceinline__ void inv_group_last_scaled(double (&v)[16], int b0, int logN, const F64LazyArith& ar) {
#pragma unroll
  for (int j = 0; j < G - 1; j++) {
    const int half = 1 << j;
#pragma unroll
    for (int r = 0; r < (1 << G); r++) {
      if (r & half) continue;
      const u32 widx = (1u << (logN - 1 - b0 - j)) + (u32)(r >> (j + 1));
      const double U = v[r], V = v[r + half];
      v[r] = U + V;
      v[r + half] = f64_mulmod_signed(U - V, ar.w[widx], ar.q, ar.qinv);
    }
  }
  // the last stage: logN - 1 - b0 - (G - 1) = 0, twiddle index 1
  const double wn = f64_canon(f64_mulmod_signed(ar.w[1], ar.ninv, ar.q, ar.qinv), ar.q, ar.qinv);
  constexpr int half = 1 << (G - 1);
#pragma unroll
  for (int r = 0; r < half; r++) {
    const double U = v[r], V = v[r + half];
    v[r] = f64_mulmod_signed(U + V, ar.ninv, ar.q, ar.qinv);
    v[r + half] = f64_mulmod_signed(U - V, wn, ar.q, ar.qinv);
  }
}

#define TILE 4096
// LDS index of (row r, column c) in the column pass, C columns per tile
__device__ __forceinline__ int lds_rc(int r, int c, int C) { return r * (C + 1) + c; }
// LDS index of (block b, element e) in the block pass, T1 words per block
__device__ __forceinline__ int lds_be(int b, int e, int T1) { return b * (T1 + (T1 >> 4) + 1) + e + (e >> 4); }
#define LDS_WORDS (TILE + TILE / 16 + 64)

// Loads of the forward column pass: the limb itself, or a value computed
// from other limbs at the same coefficient (ModupLoad).
struct LoadPlain {
  typedef u64 Raw;
  const u64* a;
  __device__ __forceinline__ void raw(size_t idx, Raw& r) const { r = a[idx]; }
  __device__ __forceinline__ u64 fin_u(const Raw& r) const { return r; }
};
// Loaders work in two phases so that the loads of a batch of values are all
// in flight before any is used: raw() issues the loads, fin_u() gives the
// residue in [0, q); loaders for the lazy FP64 arithmetic also give a centred
// double (fin_d, |value| <= q / 2 + 1), which it takes as it is.
template <class A, class LD>
__device__ __forceinline__ typename A::V fin(const A& ar, const LD& ld, const typename LD::Raw& r) {
  return ar.load(ld.fin_u(r));
}
template <int NB, class A, class LD>
__device__ __forceinline__ void fetch_batch(const A& ar, const LD& ld, const size_t (&idx)[NB], typename A::V* out) {
  typename LD::Raw raw[NB];
#pragma unroll
  for (int e = 0; e < NB; e++) ld.raw(idx[e], raw[e]);
#pragma unroll
  for (int e = 0; e < NB; e++) out[e] = fin(ar, ld, raw[e]);
}

// Forward column pass of one tile by TPB threads (tid < TPB; every thread of
// the work-group reaches its one barrier); store = false computes without
// writing (a work-group half with nothing to do).
template <int LOGN, int GA, int GB, class A, class LD>
__device__ __forceinline__ void ntt_cols2_fwd(u64* a, int c0, typename A::V* sh, const A& ar, const LD& ld, int tid,
                                              bool store) {
  typedef typename A::V V;
  constexpr int S1 = GA + GB, R = 1 << S1, T1 = (1 << LOGN) / R, C = TILE / R;
  V v[16];
  // group A: r bits [GB, S1) -> stages 0..GA-1
  constexpr int ITA = 16 >> GA;
#pragma unroll
  for (int k = 0; k < ITA; k++) {
    const int it = tid + TPB * k, c = it % C, rl = it / C;
    constexpr int NB = (1 << GA) < 8 ? (1 << GA) : 8;
#pragma unroll
    for (int h = 0; h < (1 << GA) / NB; h++) {
      size_t idx[NB];
#pragma unroll
      for (int e = 0; e < NB; e++) idx[e] = (size_t)(rl + ((h * NB + e) << GB)) * T1 + c0 + c;
      fetch_batch<NB>(ar, ld, idx, v + h * NB);
    }
    fwd_group<GA>(v, 0, 0u, ar);
#pragma unroll
    for (int mm = 0; mm < (1 << GA); mm++) sh[lds_rc(rl + (mm << GB), c, C)] = v[mm];
  }
  __syncthreads();
  // group B: r bits [0, GB) -> stages GA..S1-1
  constexpr int ITB = 16 >> GB;
#pragma unroll
  for (int k = 0; k < ITB; k++) {
    const int it = tid + TPB * k, c = it % C, rh = it / C;
#pragma unroll
    for (int mm = 0; mm < (1 << GB); mm++) v[mm] = sh[lds_rc((rh << GB) + mm, c, C)];
    fwd_group<GB>(v, GA, (u32)rh, ar);
    if (store)
#pragma unroll
      for (int mm = 0; mm < (1 << GB); mm++) a[(size_t)((rh << GB) + mm) * T1 + c0 + c] = ar.store(v[mm]);
  }
}

// Column pass body: rows R = 2^(GA+GB), C = TILE / R columns per work-group.
template <int LOGN, int GA, int GB, bool INV, class A, class LD>
__device__ __forceinline__ void ntt_cols2_body(u64* a, int c0, typename A::V* sh, const A& ar, const LD& ld) {
  typedef typename A::V V;
  constexpr int S1 = GA + GB, R = 1 << S1, T1 = (1 << LOGN) / R, C = TILE / R;
  const int tid = threadIdx.x;
  V v[16];
  if (!INV) {
    ntt_cols2_fwd<LOGN, GA, GB>(a, c0, sh, ar, ld, tid, true);
  } else {
    constexpr int S2 = LOGN - S1;
    // inverse bits [S2, S2+GB) = r bits [0, GB)
    constexpr int ITB = 16 >> GB;
#pragma unroll
    for (int k = 0; k < ITB; k++) {
      const int it = tid + TPB * k, c = it % C, rh = it / C;
#pragma unroll
      for (int mm = 0; mm < (1 << GB); mm++) v[mm] = ar.load(a[(size_t)((rh << GB) + mm) * T1 + c0 + c]);
      inv_group<GB>(v, S2, LOGN, (u32)rh, ar);
#pragma unroll
      for (int mm = 0; mm < (1 << GB); mm++) sh[lds_rc((rh << GB) + mm, c, C)] = v[mm];
    }
    __syncthreads();
    // inverse bits [S2+GB, LOGN) = r bits [GB, S1), then N^{-1}
    constexpr int ITA = 16 >> GA;
#pragma unroll
    for (int k = 0; k < ITA; k++) {
      const int it = tid + TPB * k, c = it % C, rl = it / C;
#pragma unroll
      for (int mm = 0; mm < (1 << GA); mm++) v[mm] = ar.reduce(sh[lds_rc(rl + (mm << GB), c, C)]);
      inv_group_last_scaled<GA>(v, S2 + GB, LOGN, ar);
#pragma unroll
      for (int mm = 0; mm < (1 << GA); mm++) a[(size_t)(rl + (mm << GB)) * T1 + c0 + c] = ar.store(v[mm]);
    }
  }
}

// Stores of the forward block pass: the transform itself, or (SubScale)
// out = (x - y) c mod q, the tail of ModDown (c = P^-1) and of Rescale
// (c = q_l^-1), so that y never returns to memory.
template <class A>
struct StorePlain {
  u64* a;
  const A& ar;
  __device__ __forceinline__ void pre() {}
  __device__ __forceinline__ void operator()(int e, int k, typename A::V v) const { a[e] = ar.store(v); }
};
// Decomposition digits on moduli below 2^46 are kept as the bit pattern of a
// double holding a centred representative (|v| <= q/2 + 1), the operand form
// of the key inner products; other limbs hold residues in [0, q).
struct StoreCentred {
  u64* a;
  const F64LazyArith& ar;
  __device__ __forceinline__ void pre() {}
  __device__ __forceinline__ void operator()(int e, int k, double v) const {
    a[e] = (u64)__double_as_longlong(ar.reduce(v));
  }
};
// x is read into registers when the pass starts (pre), so its loads are in
// flight during the butterflies; element e = threadIdx.x + k TPB
struct SubScaleShoup {
  u64* out;
  const u64* __restrict__ x;
  u64 c, c_sh, q;
  u64 xv[TILE / TPB];
  __device__ __forceinline__ void pre() {
#pragma unroll
    for (int k = 0; k < TILE / TPB; k++) xv[k] = x[threadIdx.x + k * TPB];
  }
  __device__ __forceinline__ void operator()(int e, int k, u64 v) const {
    out[e] = shoup_mul(sub_mod(xv[k], v, q), c, c_sh, q);
  }
};
struct SubScaleF64 {
  u64* out;
  const u64* __restrict__ x;
  double c, q, qinv;
  u64 xv[TILE / TPB];
  __device__ __forceinline__ void pre() {
#pragma unroll
    for (int k = 0; k < TILE / TPB; k++) xv[k] = x[threadIdx.x + k * TPB];
  }
  // v below 9 q in absolute value (eight forward stages): |x - v| < 10 q
  __device__ __forceinline__ void operator()(int e, int k, double v) const {
    out[e] = d2u(f64_canon(f64_mulmod_signed(u2d(xv[k]) - v, c, q, qinv), q, qinv));
  }
};
// the same with the output limb stored packed (the layout LoadPacked reads;
// HB high bytes)
template <int HB>
struct SubScalePackedF64 {
  u32* lo;
  void* hi;
  const u64* __restrict__ x;
  double c, q, qinv;
  u64 xv[TILE / TPB];
  __device__ __forceinline__ void pre() {
#pragma unroll
    for (int k = 0; k < TILE / TPB; k++) xv[k] = x[threadIdx.x + k * TPB];
  }
  __device__ __forceinline__ void operator()(int e, int k, double v) const {
    const u64 w = d2u(f64_canon(f64_mulmod_signed(u2d(xv[k]) - v, c, q, qinv), q, qinv));
    lo[e] = (u32)w;
    if (HB == 1) static_cast<u8*>(hi)[e] = (u8)(w >> 32);
    else static_cast<u16*>(hi)[e] = (u16)(w >> 32);
  }
};

// Block pass body: blocks of T1 = 2^(GC+GD) words, K = TILE / T1 blocks per work-group.
// Loads of the forward block pass: the limb's words, or (LoadPacked) the
// 32-bit plane and the high plane of a limb stored packed.
struct LoadWords {
  template <class A>
  __device__ __forceinline__ typename A::V operator()(const u64* a, size_t idx, const A& ar) const {
    return ar.load(a[idx]);
  }
};
// the words of another array at the same place (an out-of-place pass)
struct LoadFrom {
  const u64* p;
  template <class A>
  __device__ __forceinline__ typename A::V operator()(const u64*, size_t idx, const A& ar) const {
    return ar.load(p[idx]);
  }
};
// Limbs of FP64 moduli (below 2^46) stored packed within their N-word slot:
// the low 32 bits of every residue first (4N bytes), then the high bits, one
// byte each for moduli of at most 40 bits (HB = 1), two bytes otherwise.
template <int HB>
struct LoadPacked {
  const u32* lo;
  const void* hi;
  template <class A>
  __device__ __forceinline__ typename A::V operator()(const u64*, size_t idx, const A& ar) const {
    const u64 h = HB == 1 ? (u64) static_cast<const u8*>(hi)[idx] : (u64) static_cast<const u16*>(hi)[idx];
    return ar.load((u64)lo[idx] | (h << 32));
  }
};
template <int LOGN, int GC, int GD, bool INV, class A, class ST, class YL = LoadWords>
__device__ __forceinline__ void ntt_rows2_body(u64* a, int blk0, typename A::V* sh, const A& ar, ST st,
                                               const YL& yl = YL()) {
  typedef typename A::V V;
  constexpr int S2 = GC + GD, T1 = 1 << S2, S1 = LOGN - S2;
  const int tid = threadIdx.x;
  constexpr int LOWC = 1 << (S2 - GC);  // e bits below group C
  V v[16];
  if (!INV) {
    st.pre();
    // group C: e bits [GD, S2) -> stages S1..S1+GC-1
    constexpr int ITC = 16 >> GC;
#pragma unroll
    for (int k = 0; k < ITC; k++) {
      const int it = tid + TPB * k, el = it % LOWC, b = it / LOWC;
#pragma unroll
      for (int mm = 0; mm < (1 << GC); mm++) v[mm] = yl(a, (size_t)b * T1 + el + (mm << GD), ar);
      fwd_group<GC>(v, S1, (u32)(blk0 + b), ar);
#pragma unroll
      for (int mm = 0; mm < (1 << GC); mm++) sh[lds_be(b, el + (mm << GD), T1)] = v[mm];
    }
    __syncthreads();
    // group D: e bits [0, GD) -> stages S1+GC..LOGN-1
    constexpr int ITD = 16 >> GD;
    constexpr int HIGHD = 1 << (S2 - GD);
#pragma unroll
    for (int k = 0; k < ITD; k++) {
      const int it = tid + TPB * k, eh = it % HIGHD, b = it / HIGHD;
#pragma unroll
      for (int mm = 0; mm < (1 << GD); mm++) v[mm] = sh[lds_be(b, (eh << GD) + mm, T1)];
      fwd_group_last<GD>(v, S1 + GC, (u32)(((blk0 + b) << GC) + eh), ar);
#pragma unroll
      for (int mm = 0; mm < (1 << GD); mm++) sh[lds_be(b, (eh << GD) + mm, T1)] = v[mm];
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < TILE / TPB; k++) {
      const int e = tid + k * TPB;
      st(e, k, sh[lds_be(e / T1, e % T1, T1)]);
    }
  } else {
    // inverse bits [0, GD) of e
    constexpr int ITD = 16 >> GD;
    constexpr int HIGHD = 1 << (S2 - GD);
    // all sixteen loads of a thread in flight before the first LDS store
    static_assert(TILE / TPB == 16, "one register per coefficient of a thread");
#pragma unroll
    for (int k = 0; k < TILE / TPB; k++) v[k] = yl(a, tid + k * TPB, ar);
#pragma unroll
    for (int k = 0; k < TILE / TPB; k++) {
      const int e = tid + k * TPB;
      sh[lds_be(e / T1, e % T1, T1)] = v[k];
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < ITD; k++) {
      const int it = tid + TPB * k, eh = it % HIGHD, b = it / HIGHD;
#pragma unroll
      for (int mm = 0; mm < (1 << GD); mm++) v[mm] = sh[lds_be(b, (eh << GD) + mm, T1)];
      inv_group_first<GD>(v, LOGN, (u32)(((blk0 + b) << GC) + eh), ar);
#pragma unroll
      for (int mm = 0; mm < (1 << GD); mm++) sh[lds_be(b, (eh << GD) + mm, T1)] = v[mm];
    }
    __syncthreads();
    // inverse bits [GD, S2) of e
    constexpr int ITC = 16 >> GC;
#pragma unroll
    for (int k = 0; k < ITC; k++) {
      const int it = tid + TPB * k, el = it % LOWC, b = it / LOWC;
#pragma unroll
      for (int mm = 0; mm < (1 << GC); mm++) v[mm] = ar.reduce(sh[lds_be(b, el + (mm << GD), T1)]);
      inv_group<GC>(v, GD, LOGN, (u32)(blk0 + b), ar);
#pragma unroll
      for (int mm = 0; mm < (1 << GC); mm++) a[(size_t)b * T1 + el + (mm << GD)] = ar.store(v[mm]);
    }
  }
}

// moduli below 2^46 take the lazy FP64 arithmetic

template <int LOGN, int GA, int GB, bool INV>
__global__ void __launch_bounds__(TPB) k_ntt_cols2(u64* data, LimbMap map, const u64* __restrict__ tw,
                                                   const u64* __restrict__ twsh, const double* __restrict__ twf,
                                                   const ModConst* __restrict__ mc) {
  constexpr int S1 = GA + GB, R = 1 << S1, C = TILE / R;
  __shared__ u64 sh[LDS_WORDS];
  const int limb = blockIdx.y;
  const int m = limb_mod(map, limb);
  if (m < 0) return;
  const u64 N = 1ull << LOGN;
  u64* a = data + limb_slot(map, limb) * N;
  const int c0 = blockIdx.x * C;
  const ModConst mk = mc[m];
  if (mk.bits <= F64_LAZY_BITS) {
    F64LazyArith ar{twf + (size_t)m * N, mk.qf, mk.qinvf, (double)mk.ninv};
    ntt_cols2_body<LOGN, GA, GB, INV>(a, c0, reinterpret_cast<double*>(sh), ar, LoadPlain{a});
  } else {
    ShoupArith ar{tw + (size_t)m * N, twsh + (size_t)m * N, mk.q, mk.ninv, mk.ninv_sh};
    ntt_cols2_body<LOGN, GA, GB, INV>(a, c0, sh, ar, LoadPlain{a});
  }
}

// DIG: the forward pass of a decomposition, F64 limbs stored centred as doubles
template <int LOGN, int GC, int GD, bool INV, bool DIG = false>
__global__ void __launch_bounds__(TPB) k_ntt_rows2(u64* data, LimbMap map, const u64* __restrict__ tw,
                                                   const u64* __restrict__ twsh, const double* __restrict__ twf,
                                                   const ModConst* __restrict__ mc, int il) {
  constexpr int S2 = GC + GD, T1 = 1 << S2, K = TILE / T1;
  __shared__ u64 sh[LDS_WORDS];
  const int limb = grid_limb(blockIdx.y, il);
  const int m = limb_mod(map, limb);
  if (m < 0) return;
  const u64 N = 1ull << LOGN;
  const int blk0 = blockIdx.x * K;
  u64* a = data + limb_slot(map, limb) * N + (size_t)blk0 * T1;
  const ModConst mk = mc[m];
  if (mk.bits <= F64_LAZY_BITS) {
    F64LazyArith ar{twf + (size_t)m * N, mk.qf, mk.qinvf, (double)mk.ninv};
    if (DIG)
      ntt_rows2_body<LOGN, GC, GD, INV>(a, blk0, reinterpret_cast<double*>(sh), ar, StoreCentred{a, ar});
    else
      ntt_rows2_body<LOGN, GC, GD, INV>(a, blk0, reinterpret_cast<double*>(sh), ar, StorePlain<F64LazyArith>{a, ar});
  } else {
    ShoupArith ar{tw + (size_t)m * N, twsh + (size_t)m * N, mk.q, mk.ninv, mk.ninv_sh};
    ntt_rows2_body<LOGN, GC, GD, INV>(a, blk0, sh, ar, StorePlain<ShoupArith>{a, ar});
  }
}

// The inverse passes over limbs of many elements (launch_intt_many): the
// kernels of k_ntt_rows2 / k_ntt_cols2 with the limb's address taken from a
// table of element bases
struct LimbBases {
  u64* base[MR_MAX];
  int per_elem, per, stride, off;
};
__device__ __forceinline__ u64* limb_base_addr(const LimbBases& lb, int k, u64 N) {
  const int e = k / lb.per_elem, j = k - e * lb.per_elem;
  return lb.base[e] + ((size_t)(j / lb.per) * lb.stride + lb.off + j % lb.per) * N;
}
template <int LOGN, int GA, int GB>
__global__ void __launch_bounds__(TPB) k_intt_cols2_many(LimbBases lb, LimbMap map, const u64* __restrict__ tw,
                                                         const u64* __restrict__ twsh, const double* __restrict__ twf,
                                                         const ModConst* __restrict__ mc) {
  constexpr int S1 = GA + GB, R = 1 << S1, C = TILE / R;
  __shared__ u64 sh[LDS_WORDS];
  const int limb = blockIdx.y;
  const int m = limb_mod(map, limb);
  if (m < 0) return;
  const u64 N = 1ull << LOGN;
  u64* a = limb_base_addr(lb, limb, N);
  const int c0 = blockIdx.x * C;
  const ModConst mk = mc[m];
  if (mk.bits <= F64_LAZY_BITS) {
    F64LazyArith ar{twf + (size_t)m * N, mk.qf, mk.qinvf, (double)mk.ninv};
    ntt_cols2_body<LOGN, GA, GB, true>(a, c0, reinterpret_cast<double*>(sh), ar, LoadPlain{a});
  } else {
    ShoupArith ar{tw + (size_t)m * N, twsh + (size_t)m * N, mk.q, mk.ninv, mk.ninv_sh};
    ntt_cols2_body<LOGN, GA, GB, true>(a, c0, sh, ar, LoadPlain{a});
  }
}
template <int LOGN, int GC, int GD>
__global__ void __launch_bounds__(TPB) k_intt_rows2_many(LimbBases lb, LimbMap map, const u64* __restrict__ tw,
                                                         const u64* __restrict__ twsh, const double* __restrict__ twf,
                                                         const ModConst* __restrict__ mc, int il) {
  constexpr int S2 = GC + GD, T1 = 1 << S2, K = TILE / T1;
  __shared__ u64 sh[LDS_WORDS];
  const int limb = grid_limb(blockIdx.y, il);
  const int m = limb_mod(map, limb);
  if (m < 0) return;
  const u64 N = 1ull << LOGN;
  const int blk0 = blockIdx.x * K;
  u64* a = limb_base_addr(lb, limb, N) + (size_t)blk0 * T1;
  const ModConst mk = mc[m];
  if (mk.bits <= F64_LAZY_BITS) {
    F64LazyArith ar{twf + (size_t)m * N, mk.qf, mk.qinvf, (double)mk.ninv};
    ntt_rows2_body<LOGN, GC, GD, true>(a, blk0, reinterpret_cast<double*>(sh), ar, StorePlain<F64LazyArith>{a, ar});
  } else {
    ShoupArith ar{tw + (size_t)m * N, twsh + (size_t)m * N, mk.q, mk.ninv, mk.ninv_sh};
    ntt_rows2_body<LOGN, GC, GD, true>(a, blk0, sh, ar, StorePlain<ShoupArith>{a, ar});
  }
}

// Forward block pass whose stores are the SubScale tail: data holds npoly x
// nq limbs y (column pass done), x [npoly][x_stride][N], c pairs (value,
// Shoup companion) per limb t < nq, out [npoly][nq][N].
template <int LOGN, int GC, int GD>
__global__ void __launch_bounds__(TPB) k_ntt_rows2_sub(u64* data, LimbMap map, const u64* __restrict__ tw,
                                                       const u64* __restrict__ twsh, const double* __restrict__ twf,
                                                       const ModConst* __restrict__ mc, int nq,
                                                       const u64* __restrict__ x, int x_stride,
                                                       const u64* __restrict__ cpairs, u64* out, int il,
                                                       int packed, int pack_out) {
  constexpr int S2 = GC + GD, T1 = 1 << S2, K = TILE / T1;
  __shared__ u64 sh[LDS_WORDS];
  const int limb = grid_limb(blockIdx.y, il);
  const int m = limb_mod(map, limb);
  if (m < 0) return;
  const int p = limb / nq, t = limb - p * nq;
  const u64 N = 1ull << LOGN;
  const int blk0 = blockIdx.x * K;
  const size_t off = (size_t)blk0 * T1;
  u64* a = data + (size_t)limb * N + off;
  const u64* xa = x + ((size_t)p * x_stride + t) * N + off;
  u64* oa = out + ((size_t)p * nq + t) * N + off;
  const ModConst mk = mc[m];
  if (mk.bits <= F64_LAZY_BITS) {
    F64LazyArith ar{twf + (size_t)m * N, mk.qf, mk.qinvf, (double)mk.ninv};
    const SubScaleF64 st{oa, xa, u2d(cpairs[2 * t]), mk.qf, mk.qinvf};
    if (pack_out) {
      // the output limb packed too (read back by the tensor sums)
      u32* olo = reinterpret_cast<u32*>(out + ((size_t)p * nq + t) * N);
      auto go = [&](auto sto) {
        if (packed && mk.bits <= 40)
          ntt_rows2_body<LOGN, GC, GD, false>(
              a, blk0, reinterpret_cast<double*>(sh), ar, sto,
              LoadPacked<1>{reinterpret_cast<const u32*>(data + (size_t)limb * N) + off,
                            reinterpret_cast<const u8*>(reinterpret_cast<const u32*>(data + (size_t)limb * N) + N) + off});
        else if (packed)
          ntt_rows2_body<LOGN, GC, GD, false>(
              a, blk0, reinterpret_cast<double*>(sh), ar, sto,
              LoadPacked<2>{reinterpret_cast<const u32*>(data + (size_t)limb * N) + off,
                            reinterpret_cast<const u16*>(reinterpret_cast<const u32*>(data + (size_t)limb * N) + N) + off});
        else
          ntt_rows2_body<LOGN, GC, GD, false>(a, blk0, reinterpret_cast<double*>(sh), ar, sto);
      };
      if (mk.bits <= 40)
        go(SubScalePackedF64<1>{olo + off, reinterpret_cast<u8*>(olo + N) + off, xa, u2d(cpairs[2 * t]), mk.qf,
                                mk.qinvf});
      else
        go(SubScalePackedF64<2>{olo + off, reinterpret_cast<u16*>(olo + N) + off, xa, u2d(cpairs[2 * t]), mk.qf,
                                mk.qinvf});
    } else if (packed) {
      // y of this limb packed by the column pass (the int8 lift's)
      const u32* lo = reinterpret_cast<const u32*>(data + (size_t)limb * N);
      if (mk.bits <= 40)
        ntt_rows2_body<LOGN, GC, GD, false>(a, blk0, reinterpret_cast<double*>(sh), ar, st,
                                            LoadPacked<1>{lo + off, reinterpret_cast<const u8*>(lo + N) + off});
      else
        ntt_rows2_body<LOGN, GC, GD, false>(a, blk0, reinterpret_cast<double*>(sh), ar, st,
                                            LoadPacked<2>{lo + off, reinterpret_cast<const u16*>(lo + N) + off});
    } else {
      ntt_rows2_body<LOGN, GC, GD, false>(a, blk0, reinterpret_cast<double*>(sh), ar, st);
    }
  } else {
    ShoupArith ar{tw + (size_t)m * N, twsh + (size_t)m * N, mk.q, mk.ninv, mk.ninv_sh};
    ntt_rows2_body<LOGN, GC, GD, false>(a, blk0, sh, ar, SubScaleShoup{oa, xa, cpairs[2 * t], cpairs[2 * t + 1], mk.q});
  }
}

// Decompose with the basis conversion fused into the forward column pass:
// the value of digit j at modulus m and coefficient i is
//   sum_a y_a[i] hat_(a,m) mod q_m,  y_a = coefficient-domain source limb a of
// digit j already multiplied by its hat inverse,
// computed while loading the pass's tile (no converted limb goes to memory).
// The digit's own limbs copy the evaluation-domain input instead.
struct ModupSrc {
  const u64* y;       // [B][nq][N]
  const u64* ntt_in;  // [B][nq][N]
  int nq, nqp, alpha, beta, L;
  int ns[16], srcbits[16];
  const u64* hat_t[16];     // [ns][nmods]
  const u64* hat_t_sh[16];
};
// F64: every source below 4 q (signed exact products, one reduction);
// otherwise Shoup products.  The source loop has a compile-time length NS
// without branches: 3 for a full digit of three limbs, else 4 with sources
// past ns repeating the last one against zero constants; so the loads of a
// tile's values can all be in flight together.
struct ModupData {
  const u64* y0;
  u64 N;
  int ns;
  u64 q, h[4], hs[4];
  double qf, qinvf, hf[4];
};
template <bool F64, int NS = 4>
struct ModupLoad : ModupData {
  struct Raw {
    u64 x[NS];
  };
  __device__ __forceinline__ void raw(size_t idx, Raw& r) const {
#pragma unroll
    for (int a = 0; a < NS; a++) r.x[a] = y0[(size_t)(a < ns ? a : ns - 1) * N + idx];
  }
  __device__ __forceinline__ double sum_f64(const Raw& r) const {
    double acc = 0.0;
#pragma unroll
    for (int a = 0; a < NS; a++) acc += f64_mulmod_signed(u2d(r.x[a]), hf[a], qf, qinvf);
    return acc;
  }
  __device__ __forceinline__ u64 fin_u(const Raw& r) const {
    if (F64) return d2u(f64_canon(sum_f64(r), qf, qinvf));
    u64 acc = 0;
#pragma unroll
    for (int a = 0; a < NS; a++) acc = add_mod(acc, shoup_mul(r.x[a], h[a], hs[a], q), q);
    return acc;
  }
  __device__ __forceinline__ double fin_d(const Raw& r) const { return f64_centre(sum_f64(r), qf, qinvf); }
};
template <int NS>
__device__ __forceinline__ double fin(const F64LazyArith&, const ModupLoad<true, NS>& ld,
                                      const typename ModupLoad<true, NS>::Raw& r) {
  return ld.fin_d(r);
}
template <class L>
__device__ __forceinline__ L loader_of(const ModupData& d) {
  L l;
  static_cast<ModupData&>(l) = d;
  return l;
}
template <int LOGN, int GA, int GB>
__global__ void __launch_bounds__(TPB) k_ntt_cols2_modup(u64* digits, ModupSrc S, const u64* __restrict__ tw,
                                                         const u64* __restrict__ twsh,
                                                         const double* __restrict__ twf, int nmods,
                                                         const ModConst* __restrict__ mc) {
  constexpr int S1 = GA + GB, R = 1 << S1, T1 = (1 << LOGN) / R, C = TILE / R;
  __shared__ u64 sh[LDS_WORDS];
  const int limb = blockIdx.y;
  const int per = S.beta * S.nqp;
  const int b = limb / per, rem = limb - b * per, j = rem / S.nqp, pos = rem - j * S.nqp;
  const u64 N = 1ull << LOGN;
  u64* a = digits + (size_t)limb * N;
  const int c0 = blockIdx.x * C;
  if (pos < S.nq && pos / S.alpha == j) {
    // the digit's own limbs: the input itself (centred doubles on F64 moduli)
    const u64* src = S.ntt_in + ((size_t)b * S.nq + pos) * N;
    const bool f64 = mc[pos].bits <= F64_LAZY_BITS;
    u64 t[TILE / TPB];
#pragma unroll
    for (int k = 0; k < TILE / TPB; k++) {
      const int e = threadIdx.x + k * TPB;
      t[k] = src[(size_t)(e / C) * T1 + c0 + e % C];
    }
#pragma unroll
    for (int k = 0; k < TILE / TPB; k++) {
      const int e = threadIdx.x + k * TPB;
      a[(size_t)(e / C) * T1 + c0 + e % C] = f64 ? (u64)__double_as_longlong(u2d(t[k])) : t[k];
    }
    return;
  }
  const int m = pos < S.nq ? pos : S.L + 1 + (pos - S.nq);
  const ModConst mk = mc[m];
  ModupData d;
  d.y0 = S.y + ((size_t)b * S.nq + (size_t)j * S.alpha) * N;
  d.N = N;
  d.ns = S.ns[j];
  d.q = mk.q;
  d.qf = mk.qf;
  d.qinvf = mk.qinvf;
  for (int x = 0; x < 4; x++) {
    const bool in = x < d.ns;
    d.h[x] = in ? S.hat_t[j][(size_t)x * nmods + m] : 0;
    d.hs[x] = in ? S.hat_t_sh[j][(size_t)x * nmods + m] : 0;
    d.hf[x] = u2d(d.h[x]);
  }
  if (mk.bits <= F64_LAZY_BITS) {
    F64LazyArith ar{twf + (size_t)m * N, mk.qf, mk.qinvf, (double)mk.ninv};
    double* shd = reinterpret_cast<double*>(sh);
    if (S.srcbits[j] > (int)mk.bits + 1)
      ntt_cols2_body<LOGN, GA, GB, false>(a, c0, shd, ar, loader_of<ModupLoad<false>>(d));
    else if (d.ns == 3)  // a full digit of three limbs: no padding source
      ntt_cols2_body<LOGN, GA, GB, false>(a, c0, shd, ar, loader_of<ModupLoad<true, 3>>(d));
    else
      ntt_cols2_body<LOGN, GA, GB, false>(a, c0, shd, ar, loader_of<ModupLoad<true>>(d));
  } else {
    ShoupArith ar{tw + (size_t)m * N, twsh + (size_t)m * N, mk.q, mk.ninv, mk.ninv_sh};
    ntt_cols2_body<LOGN, GA, GB, false>(a, c0, sh, ar, loader_of<ModupLoad<false>>(d));
  }
}

template <int LOGN, int GA, int GB, int GC, int GD>
static void ntt2_modup(const DeviceTables& T, u64* digits, const ModupSrc& S, int batch, const LimbMap& rows_map,
                       hipStream_t s) {
  constexpr int R = 1 << (GA + GB), C = TILE / R, T1 = 1 << (GC + GD), K = TILE / T1;
  const int nlimbs = batch * S.beta * S.nqp;
  dim3 gc((1 << LOGN) / R / C, nlimbs), gr(((1 << LOGN) / T1) / K, nlimbs);
  // butterflies of the column stages on every converted digit limb, plus the
  // conversion (ns products per value); the rows pass transforms the same limbs
  Mm mm_cols;
  for (int k = 0; k < S.beta * S.nqp; k++) {
    const int idx = rows_map.idx[k];
    if (idx >= 0) mm_cols.add(T.bits[idx], batch * (0.5 * T.N * (GA + GB) + (double)T.N * S.ns[k / S.nqp]));
  }
  {
    ProfScope ps("ntt_fwd_cols_modup", s, 8.0 * T.N * batch * (2.0 * S.nq + (double)S.beta * S.nqp), mm_cols);
    hipLaunchKernelGGL((k_ntt_cols2_modup<LOGN, GA, GB>), gc, dim3(TPB), 0, s, digits, S, T.psi, T.psi_sh, T.psi_f,
                       T.nmods, T.mc);
  }
  int active = 0;
  for (int k = 0; k < rows_map.n; k++) active += rows_map.idx[k] >= 0;
  ProfScope ps("ntt_fwd_rows", s, 16.0 * T.N * batch * active,
               mm_map(T, rows_map, S.beta * S.nqp, batch * 0.5 * T.N * (GC + GD)));
  hipLaunchKernelGGL((k_ntt_rows2<LOGN, GC, GD, false, true>), gr, dim3(TPB), 0, s, digits, rows_map, T.psi,
                     T.psi_sh, T.psi_f, T.mc, interleave_of(nlimbs, modulus_period(rows_map), g_knobs.ntt_interleave));
}

template <int LOGN, int GA, int GB, int GC, int GD>
static void ntt2_fwd_sub(const DeviceTables& T, u64* y, int nq, int npoly, const LimbMap& map, const u64* x,
                         int x_stride, const u64* cpairs, u64* out, hipStream_t s, bool do_cols = true,
                         bool packed = false, bool pack_out = false) {
  constexpr int R = 1 << (GA + GB), C = TILE / R, T1 = 1 << (GC + GD), K = TILE / T1;
  const int nlimbs = nq * npoly;
  dim3 gc((1 << LOGN) / R / C, nlimbs), gr(((1 << LOGN) / T1) / K, nlimbs);
  if (do_cols) {
    ProfScope ps("ntt_fwd_cols", s, 16.0 * nlimbs * T.N, mm_map(T, map, nlimbs, 0.5 * T.N * (GA + GB)));
    hipLaunchKernelGGL((k_ntt_cols2<LOGN, GA, GB, false>), gc, dim3(TPB), 0, s, y, map, T.psi, T.psi_sh, T.psi_f,
                       T.mc);
  }
  ProfScope ps("ntt_fwd_rows_sub", s, 24.0 * nlimbs * T.N, mm_map(T, map, nlimbs, 0.5 * T.N * (GC + GD) + T.N));
  hipLaunchKernelGGL((k_ntt_rows2_sub<LOGN, GC, GD>), gr, dim3(TPB), 0, s, y, map, T.psi, T.psi_sh, T.psi_f, T.mc,
                     nq, x, x_stride, cpairs, out, interleave_of(nlimbs, modulus_period(map), g_knobs.ntt_interleave),
                     packed ? 1 : 0, pack_out ? 1 : 0);
}

template <int LOGN, int GA, int GB, int GC, int GD>
static void ntt2(const DeviceTables& T, u64* data, int nlimbs, const LimbMap& map, bool inverse, double pass_bytes,
                 hipStream_t s) {
  constexpr int R = 1 << (GA + GB), C = TILE / R, T1 = 1 << (GC + GD), K = TILE / T1;
  static_assert(GA + GB + GC + GD == LOGN, "stage split");
  dim3 gc((1 << LOGN) / R / C, nlimbs), gr(((1 << LOGN) / T1) / K, nlimbs);
  const int il = interleave_of(nlimbs, modulus_period(map), g_knobs.ntt_interleave);
  const Mm mm_c = mm_map(T, map, nlimbs, 0.5 * T.N * (GA + GB)), mm_r = mm_map(T, map, nlimbs, 0.5 * T.N * (GC + GD));
  if (!inverse) {
    {
      ProfScope ps("ntt_fwd_cols", s, pass_bytes, mm_c);
      hipLaunchKernelGGL((k_ntt_cols2<LOGN, GA, GB, false>), gc, dim3(TPB), 0, s, data, map, T.psi, T.psi_sh,
                         T.psi_f, T.mc);
    }
    ProfScope ps("ntt_fwd_rows", s, pass_bytes, mm_r);
    hipLaunchKernelGGL((k_ntt_rows2<LOGN, GC, GD, false>), gr, dim3(TPB), 0, s, data, map, T.psi, T.psi_sh,
                       T.psi_f, T.mc, il);
  } else {
    {
      ProfScope ps("ntt_inv_rows", s, pass_bytes, mm_r);
      hipLaunchKernelGGL((k_ntt_rows2<LOGN, GC, GD, true>), gr, dim3(TPB), 0, s, data, map, T.ipsi, T.ipsi_sh,
                         T.ipsi_f, T.mc, il);
    }
    ProfScope ps("ntt_inv_cols", s, pass_bytes, mm_c);
    hipLaunchKernelGGL((k_ntt_cols2<LOGN, GA, GB, true>), gc, dim3(TPB), 0, s, data, map, T.ipsi, T.ipsi_sh,
                       T.ipsi_f, T.mc);
  }
}


// Inverse NTT from src into data whose last stage scales limb k by
// scales[2 m] (Shoup pair; m its modulus) in place of N^-1: Decompose's
// coefficient-domain sources times their hat inverses, from the input limbs.
template <int LOGN, int GC, int GD>
__global__ void __launch_bounds__(TPB) k_intt_rows2_src(u64* data, const u64* __restrict__ src, LimbMap map,
                                                        const u64* __restrict__ tw, const u64* __restrict__ twsh,
                                                        const double* __restrict__ twf,
                                                        const ModConst* __restrict__ mc, int il) {
  constexpr int S2 = GC + GD, T1 = 1 << S2, K = TILE / T1;
  __shared__ u64 sh[LDS_WORDS];
  const int limb = grid_limb(blockIdx.y, il);
  const int m = limb_mod(map, limb);
  if (m < 0) return;
  const u64 N = 1ull << LOGN;
  const int blk0 = blockIdx.x * K;
  const size_t off = limb_slot(map, limb) * N + (size_t)blk0 * T1;
  u64* a = data + off;
  const ModConst mk = mc[m];
  if (mk.bits <= F64_LAZY_BITS) {
    F64LazyArith ar{twf + (size_t)m * N, mk.qf, mk.qinvf, (double)mk.ninv};
    ntt_rows2_body<LOGN, GC, GD, true>(a, blk0, reinterpret_cast<double*>(sh), ar, StorePlain<F64LazyArith>{a, ar},
                                       LoadFrom{src + off});
  } else {
    ShoupArith ar{tw + (size_t)m * N, twsh + (size_t)m * N, mk.q, mk.ninv, mk.ninv_sh};
    ntt_rows2_body<LOGN, GC, GD, true>(a, blk0, sh, ar, StorePlain<ShoupArith>{a, ar}, LoadFrom{src + off});
  }
}
template <int LOGN, int GA, int GB>
__global__ void __launch_bounds__(TPB) k_intt_cols2_scaled(u64* data, LimbMap map, const u64* __restrict__ scales,
                                                           const u64* __restrict__ tw, const u64* __restrict__ twsh,
                                                           const double* __restrict__ twf,
                                                           const ModConst* __restrict__ mc) {
  constexpr int S1 = GA + GB, R = 1 << S1, C = TILE / R;
  __shared__ u64 sh[LDS_WORDS];
  const int limb = blockIdx.y;
  const int m = limb_mod(map, limb);
  if (m < 0) return;
  const u64 N = 1ull << LOGN;
  u64* a = data + limb_slot(map, limb) * N;
  const int c0 = blockIdx.x * C;
  const ModConst mk = mc[m];
  const u64 c = scales[2 * m], csh = scales[2 * m + 1];
  if (mk.bits <= F64_LAZY_BITS) {
    F64LazyArith ar{twf + (size_t)m * N, mk.qf, mk.qinvf, (double)c};
    ntt_cols2_body<LOGN, GA, GB, true>(a, c0, reinterpret_cast<double*>(sh), ar, LoadPlain{a});
  } else {
    ShoupArith ar{tw + (size_t)m * N, twsh + (size_t)m * N, mk.q, c, csh};
    ntt_cols2_body<LOGN, GA, GB, true>(a, c0, sh, ar, LoadPlain{a});
  }
}
bool launch_intt_scaled(const DeviceTables& T, u64* data, const u64* src, int nlimbs, const LimbMap& map,
                        const u64* scales, hipStream_t s) {
  if (nlimbs <= 0) return true;
  if (map.slot_per > 0) return false;
  return ntt_dispatch(T.logN, [&](auto sp) {
    using S = decltype(sp);
    constexpr int LOGN = S::LOGN, GA = S::GA, GB = S::GB, GC = S::GC, GD = S::GD;
    constexpr int R = 1 << (GA + GB), C = TILE / R, T1 = 1 << (GC + GD), K = TILE / T1;
    dim3 gc((1 << LOGN) / R / C, nlimbs), gr(((1 << LOGN) / T1) / K, nlimbs);
    const int il = interleave_of(nlimbs, modulus_period(map), g_knobs.ntt_interleave);
    const double pass_bytes = 16.0 * nlimbs * T.N;
    {
      ProfScope ps("ntt_inv_rows", s, pass_bytes, mm_map(T, map, nlimbs, 0.5 * T.N * (GC + GD)));
      hipLaunchKernelGGL((k_intt_rows2_src<LOGN, GC, GD>), gr, dim3(TPB), 0, s, data, src, map, T.ipsi, T.ipsi_sh,
                         T.ipsi_f, T.mc, il);
    }
    ProfScope ps("ntt_inv_cols", s, pass_bytes, mm_map(T, map, nlimbs, 0.5 * T.N * (GA + GB)));
    hipLaunchKernelGGL((k_intt_cols2_scaled<LOGN, GA, GB>), gc, dim3(TPB), 0, s, data, map, scales, T.ipsi,
                       T.ipsi_sh, T.ipsi_f, T.mc);
  });
}

static bool ntt_register_blocked(const DeviceTables& T, u64* data, int nlimbs, const LimbMap& map, bool inverse,
                                 double pass_bytes, hipStream_t s) {
  return ntt_dispatch(T.logN, [&](auto sp) {
    using S = decltype(sp);
    ntt2<NTT_SPLIT_ARGS>(T, data, nlimbs, map, inverse, pass_bytes, s);
  });
}


// Each pass streams every active limb in and out once: 16 bytes per coefficient.
void launch_ntt(const DeviceTables& T, u64* data, int nlimbs, const LimbMap& map, bool inverse, hipStream_t s) {
  if (nlimbs <= 0) return;
  int active = 0;
  for (int k = 0; k < nlimbs; k++) active += map.idx[k % map.n] >= 0;
  const double pass_bytes = 16.0 * active * T.N;
  if (ntt_register_blocked(T, data, nlimbs, map, inverse, pass_bytes, s)) return;
  if (map.slot_per > 0) throw std::runtime_error("limb slots need the register-blocked NTT (log N 12..16)");
  NttShape sh = ntt_shape(T.logN);
  dim3 gc(sh.T1 / sh.C, nlimbs), gr(sh.R / sh.K, nlimbs);
  const Mm mm_c = mm_map(T, map, nlimbs, 0.5 * T.N * sh.s1), mm_r = mm_map(T, map, nlimbs, 0.5 * T.N * (sh.logN - sh.s1));
  if (!inverse) {
    {
      ProfScope ps("ntt_fwd_cols", s, pass_bytes, mm_c);
      hipLaunchKernelGGL(k_ntt_cols, gc, dim3(TPB), 0, s, data, map, sh.logN, sh.R, sh.T1, sh.C, 0, T.psi,
                         T.psi_sh, T.mc);
    }
    ProfScope ps("ntt_fwd_rows", s, pass_bytes, mm_r);
    hipLaunchKernelGGL(k_ntt_rows, gr, dim3(TPB), 0, s, data, map, sh.logN, sh.s1, sh.T1, sh.K, 0, T.psi,
                       T.psi_sh, T.mc);
  } else {
    {
      ProfScope ps("ntt_inv_rows", s, pass_bytes, mm_r);
      hipLaunchKernelGGL(k_ntt_rows, gr, dim3(TPB), 0, s, data, map, sh.logN, sh.s1, sh.T1, sh.K, 1, T.ipsi,
                         T.ipsi_sh, T.mc);
    }
    ProfScope ps("ntt_inv_cols", s, pass_bytes, mm_c);
    hipLaunchKernelGGL(k_ntt_cols, gc, dim3(TPB), 0, s, data, map, sh.logN, sh.R, sh.T1, sh.C, 1, T.ipsi,
                       T.ipsi_sh, T.mc);
  }
}

__global__ void k_moddown_final(u64* out, const u64* x, const u64* y, int nq, const u64* pinv, int x_stride_limbs,
                                int logN, const ModConst* __restrict__ mc);
// Forward NTT of npoly x nq limbs y (moduli q_0..q_{nq-1}) followed by
// out = (x - y) c mod q_t; y is left in an unspecified state.
void launch_ntt_fwd_sub(const DeviceTables& T, u64* y, int nq, int npoly, const LimbMap& map, const u64* x,
                        int x_stride, const u64* cpairs, u64* out, hipStream_t s) {
  if (nq <= 0 || npoly <= 0) return;
  if (ntt_dispatch(T.logN, [&](auto sp) {
        using S = decltype(sp);
        ntt2_fwd_sub<NTT_SPLIT_ARGS>(T, y, nq, npoly, map, x, x_stride, cpairs, out, s);
      }))
    return;
  launch_ntt(T, y, nq * npoly, map, false, s);
  dim3 grid(cdiv(T.N, TPB), nq, npoly);
  ProfScope ps("moddown_final", s, 8.0 * T.N * 3.0 * npoly * nq, mm_q(T, nq, (double)T.N, npoly));
  hipLaunchKernelGGL(k_moddown_final, grid, dim3(TPB), 0, s, out, x, y, nq, cpairs, x_stride, T.logN, T.mc);
}

// Fused ModUp + forward NTT of every digit (see k_ntt_cols2_modup); false
// when the ring size has no register-blocked NTT (the caller then converts
// and transforms separately).  y holds the sources times their hat inverses.
// digits from the generic path (residues in [0, q)) put into the key inner
// products' operand form: F64 limbs as doubles
__global__ void k_digits_f64(u64* d, LimbMap map, int logN, const ModConst* __restrict__ mc) {
  const u64 N = 1ull << logN;
  const u32 i = blockIdx.x * TPB + threadIdx.x;
  const int limb = blockIdx.y;
  const int m = limb_mod(map, limb);
  if (i >= N || m < 0 || mc[m].bits > F64_LAZY_BITS) return;
  u64* p = d + (size_t)limb * N + i;
  *p = (u64)__double_as_longlong(u2d(*p));
}
void launch_digits_f64(const DeviceTables& T, u64* d, int nlimbs, const LimbMap& map, hipStream_t s) {
  hipLaunchKernelGGL(k_digits_f64, dim3(cdiv(T.N, TPB), nlimbs), dim3(TPB), 0, s, d, map, T.logN, T.mc);
}

bool launch_modup_ntt(const DeviceTables& T, u64* digits, const u64* y, const u64* ntt_in, int level, int L,
                      int alpha, int beta, const FbcTable* tabs, int batch, const LimbMap& rows_map, hipStream_t s) {
  if (T.logN < 12 || T.logN > 16 || alpha > 4 || beta > 16) return false;
  ModupSrc S;
  S.y = y;
  S.ntt_in = ntt_in;
  S.nq = level + 1;
  S.nqp = level + 1 + alpha;
  S.alpha = alpha;
  S.beta = beta;
  S.L = L;
  for (int j = 0; j < beta; j++) {
    S.ns[j] = tabs[j].ns;
    S.srcbits[j] = 0;
    for (int a = 0; a < tabs[j].ns; a++) S.srcbits[j] = std::max(S.srcbits[j], (int)T.bits[tabs[j].src[a]]);
    S.hat_t[j] = tabs[j].hat_t;
    S.hat_t_sh[j] = tabs[j].hat_t_sh;
  }
  const ModupSrc& src = S;
  return ntt_dispatch(T.logN, [&](auto sp) {
    using S = decltype(sp);
    ntt2_modup<NTT_SPLIT_ARGS>(T, digits, src, batch, rows_map, s);
  });
}

// ---------------------------------------------------------------------------
// Galois automorphism in the evaluation domain:
//   out[i] = in[brv((g (2 brv(i) + 1) mod 2N - 1) / 2)]
// ---------------------------------------------------------------------------
__device__ __forceinline__ u32 automorph_src(u32 i, u64 g, int logN) {
  u64 twoN_mask = (2ull << logN) - 1;
  u64 e = (g * (2ull * brv(i, logN) + 1)) & twoN_mask;
  return brv((u32)((e - 1) >> 1), logN);
}

__global__ void k_automorph(u64* out, const u64* in, int nlimbs, u64 g, int logN) {
  const u64 N = 1ull << logN;
  u32 i = blockIdx.x * TPB + threadIdx.x;
  if (i >= N) return;
  u32 src = automorph_src(i, g, logN);
  for (int k = blockIdx.y; k < nlimbs; k += gridDim.y) out[(size_t)k * N + i] = in[(size_t)k * N + src];
}

void launch_automorph(const DeviceTables& T, u64* out, const u64* in, int nlimbs, u64 g, hipStream_t s) {
  dim3 grid(cdiv(T.N, TPB), nlimbs < 64 ? nlimbs : 64);
  hipLaunchKernelGGL(k_automorph, grid, dim3(TPB), 0, s, out, in, nlimbs, g, T.logN);
}

// ---------------------------------------------------------------------------
// Elementwise
// ---------------------------------------------------------------------------
enum { EW_ADD = 0, EW_SUB, EW_MUL, EW_MULACC, EW_NEG };

__global__ void k_elementwise(int op, u64* out, const u64* a, const u64* b, int nlimbs, int b_limbs, LimbMap map,
                              int logN, const ModConst* __restrict__ mc, int il) {
  const u64 N = 1ull << logN;
  int blk, k;
  block_limb(il, b_limbs, (int)(N / TPB), blk, k);
  u32 i = blk * TPB + threadIdx.x;
  if (i >= N || k >= nlimbs) return;
  int m = limb_mod(map, k);
  if (m < 0) return;
  const ModConst mk = mc[m];
  size_t o = (size_t)k * N + i;
  size_t ob = (size_t)(k % b_limbs) * N + i;
  switch (op) {
    case EW_ADD: out[o] = add_mod(a[o], b[ob], mk.q); break;
    case EW_SUB: out[o] = sub_mod(a[o], b[ob], mk.q); break;
    case EW_MUL: out[o] = mul_mod_any(a[o], b[ob], mk); break;
    case EW_MULACC: out[o] = add_mod(out[o], mul_mod_any(a[o], b[ob], mk), mk.q); break;
    case EW_NEG: out[o] = a[o] ? mk.q - a[o] : 0; break;
  }
}

static void ew(const DeviceTables& T, int op, u64* out, const u64* a, const u64* b, int nlimbs, int b_limbs,
               const LimbMap& m, hipStream_t s) {
  if (nlimbs <= 0) return;
  // reads a (and b once per distinct limb), writes out; the accumulate also reads out
  double words = (double)nlimbs * (op == EW_MULACC ? 3 : (op == EW_NEG ? 2 : 2)) + (op == EW_NEG ? 0 : b_limbs);
  ProfScope ps("elementwise", s, 8.0 * T.N * words,
               op == EW_MUL || op == EW_MULACC ? mm_map(T, m, nlimbs, (double)T.N) : Mm());
  int il;
  dim3 grid = sum_grid((int)cdiv(T.N, TPB), nlimbs, b_limbs, g_knobs.ew_interleave, il);
  hipLaunchKernelGGL(k_elementwise, grid, dim3(TPB), 0, s, op, out, a, b, nlimbs, b_limbs, m, T.logN, T.mc, il);
}
void launch_add(const DeviceTables& T, u64* out, const u64* a, const u64* b, int nl, const LimbMap& m,
                hipStream_t s) { ew(T, EW_ADD, out, a, b, nl, nl, m, s); }
void launch_sub(const DeviceTables& T, u64* out, const u64* a, const u64* b, int nl, const LimbMap& m,
                hipStream_t s) { ew(T, EW_SUB, out, a, b, nl, nl, m, s); }
void launch_mul(const DeviceTables& T, u64* out, const u64* a, const u64* b, int nl, const LimbMap& m,
                hipStream_t s) { ew(T, EW_MUL, out, a, b, nl, nl, m, s); }
void launch_mul_bcast(const DeviceTables& T, u64* out, const u64* a, const u64* b, int nl, int bl,
                      const LimbMap& m, hipStream_t s) { ew(T, EW_MUL, out, a, b, nl, bl, m, s); }
void launch_mul_acc(const DeviceTables& T, u64* acc, const u64* a, const u64* b, int nl, int bl, const LimbMap& m,
                    hipStream_t s) { ew(T, EW_MULACC, acc, a, b, nl, bl, m, s); }
// out = sum_t a_t (.) p_t (p_t broadcast with period b_limbs), one pass over
// every operand; `accumulate` adds onto out
struct SumTerms {
  const u64* a[SUM_MAX_TERMS];
  const u64* p[SUM_MAX_TERMS];
};
__global__ void k_mul_sum(u64* out, SumTerms t, int nterms, int accumulate, int b_limbs, LimbMap map, int logN,
                          const ModConst* __restrict__ mc, int il) {
  const u64 N = 1ull << logN;
  int blk, k;
  block_limb(il, b_limbs, (int)(N / TPB), blk, k);
  u32 i = blk * TPB + threadIdx.x;
  if (i >= N) return;
  int m = limb_mod(map, k);
  if (m < 0) return;
  const ModConst mk = mc[m];
  const size_t o = (size_t)k * N + i, op = (size_t)(k % b_limbs) * N + i;
  u64 an = t.a[0][o], pn = t.p[0][op];
  if (mk.bits <= F64_LAZY_BITS) {
    // up to 63 signed exact products and the old value, reduced once
    const double q = mk.qf, qi = mk.qinvf;
    double acc = accumulate ? u2d(out[o]) : 0.0;
    for (int j = 0; j < nterms; j++) {
      const u64 a = an, p = pn;
      if (j + 1 < nterms) {
        an = t.a[j + 1][o];
        pn = t.p[j + 1][op];
      }
      acc += f64_mulmod_signed(u2d(a), u2d(p), q, qi);
    }
    out[o] = d2u(f64_canon(acc, q, qi));
    return;
  }
  u64 acc = accumulate ? out[o] : 0;
  for (int j = 0; j < nterms; j++) {
    const u64 a = an, p = pn;
    if (j + 1 < nterms) {
      an = t.a[j + 1][o];
      pn = t.p[j + 1][op];
    }
    acc = add_mod(acc, mul_mod_any(a, p, mk), mk.q);
  }
  out[o] = acc;
}
void launch_mul_sum(const DeviceTables& T, u64* out, const u64* const* a, const u64* const* p, int nterms, int nl,
                    int bl, const LimbMap& m, bool accumulate, hipStream_t s) {
  // 63 terms a pass: with the old value, 64 summands below q < 2^46 each
  constexpr int TERMS = SUM_MAX_TERMS - 1;
  for (int t0 = 0; t0 < nterms; t0 += TERMS) {
    const int nt = std::min(nterms - t0, TERMS);
    const bool acc = accumulate || t0 > 0;
    SumTerms t;
    for (int j = 0; j < nt; j++) {
      t.a[j] = a[t0 + j];
      t.p[j] = p[t0 + j];
    }
    ProfScope ps("elementwise", s, 8.0 * T.N * ((double)nl * (nt + 1 + (acc ? 1 : 0)) + (double)bl * nt),
                 mm_map(T, m, nl, (double)T.N * nt));
    int il;
    dim3 grid = sum_grid((int)cdiv(T.N, TPB), nl, bl, g_knobs.ew_interleave, il);
    hipLaunchKernelGGL(k_mul_sum, grid, dim3(TPB), 0, s, out, t, nt, acc ? 1 : 0, bl, m, T.logN, T.mc, il);
  }
}

// G sums at once over shared terms: out_g = sum_t a_t (.) p_(g,t) (p_(g,t) may be
// absent); each a_t is read once for all G outputs
struct SumMulti {
  const u64* a[SUM_MAX_TERMS];
  const u64* p[SUM_MAX_OUTS][SUM_MAX_TERMS];
  u64* out[SUM_MAX_OUTS];
};
// V = 2: two consecutive coefficients per thread, 16-byte loads and stores.
// S: a thread sums S term streams that share their plaintexts (limbs k0 +
// s b_limbs, s < S, of the same modulus), loading each plaintext word once
// for all of them.
template <int G, int V, int S>
__global__ void __launch_bounds__(TPB) k_mul_sum_multi(SumMulti t, int nterms, int b_limbs, LimbMap map, int logN,
                                const ModConst* __restrict__ mc, int il) {
  const u64 N = 1ull << logN;
  int blk, k;
  block_limb(il, b_limbs, (int)(N / (TPB * V)), blk, k);
  const u32 i = (blk * TPB + threadIdx.x) * V;
  if (i >= N) return;
  const int pos = k % b_limbs, k0 = (k / b_limbs) * S * b_limbs + pos;
  int m = limb_mod(map, k0);
  if (m < 0) return;
  const ModConst mk = mc[m];
  const size_t op = (size_t)pos * N + i;
  size_t o[S];
#pragma unroll
  for (int s = 0; s < S; s++) o[s] = (size_t)(k0 + s * b_limbs) * N + i;
  struct W {
    u64 v[V];
  };
  auto ld = [](const u64* p) {
    W w;
    if (V == 2) {
      const ulonglong2 x = *reinterpret_cast<const ulonglong2*>(p);
      w.v[0] = x.x;
      w.v[V - 1] = x.y;
    } else {
      w.v[0] = *p;
    }
    return w;
  };
  // software-pipelined over the terms
  W xn[S], pn[G];
#pragma unroll
  for (int s = 0; s < S; s++) xn[s] = ld(t.a[0] + o[s]);
#pragma unroll
  for (int g = 0; g < G; g++) pn[g] = t.p[g][0] ? ld(t.p[g][0] + op) : W{};
  u64 res[G][S][V];
  if (mk.bits <= F64_LAZY_BITS) {
    // signed exact products summed per output (at most 64), reduced once
    const double q = mk.qf, qi = mk.qinvf;
    double acc[G][S][V];
#pragma unroll
    for (int g = 0; g < G; g++)
#pragma unroll
      for (int s = 0; s < S; s++)
#pragma unroll
        for (int e = 0; e < V; e++) acc[g][s][e] = 0.0;
    for (int j = 0; j < nterms; j++) {
      double x[S][V];
#pragma unroll
      for (int s = 0; s < S; s++)
#pragma unroll
        for (int e = 0; e < V; e++) x[s][e] = u2d(xn[s].v[e]);
      W pv[G];
#pragma unroll
      for (int g = 0; g < G; g++) pv[g] = pn[g];
      if (j + 1 < nterms) {
#pragma unroll
        for (int s = 0; s < S; s++) xn[s] = ld(t.a[j + 1] + o[s]);
#pragma unroll
        for (int g = 0; g < G; g++) pn[g] = t.p[g][j + 1] ? ld(t.p[g][j + 1] + op) : W{};
      }
#pragma unroll
      for (int g = 0; g < G; g++)
        if (t.p[g][j])
#pragma unroll
          for (int e = 0; e < V; e++) {
            const double pd = u2d(pv[g].v[e]);
#pragma unroll
            for (int s = 0; s < S; s++) acc[g][s][e] += f64_mulmod_signed(x[s][e], pd, q, qi);
          }
    }
#pragma unroll
    for (int g = 0; g < G; g++)
#pragma unroll
      for (int s = 0; s < S; s++)
#pragma unroll
        for (int e = 0; e < V; e++) res[g][s][e] = d2u(f64_canon(acc[g][s][e], q, qi));
  } else {
#pragma unroll
    for (int g = 0; g < G; g++)
#pragma unroll
      for (int s = 0; s < S; s++)
#pragma unroll
        for (int e = 0; e < V; e++) res[g][s][e] = 0;
    for (int j = 0; j < nterms; j++) {
      W x[S];
#pragma unroll
      for (int s = 0; s < S; s++) x[s] = xn[s];
      W pv[G];
#pragma unroll
      for (int g = 0; g < G; g++) pv[g] = pn[g];
      if (j + 1 < nterms) {
#pragma unroll
        for (int s = 0; s < S; s++) xn[s] = ld(t.a[j + 1] + o[s]);
#pragma unroll
        for (int g = 0; g < G; g++) pn[g] = t.p[g][j + 1] ? ld(t.p[g][j + 1] + op) : W{};
      }
#pragma unroll
      for (int g = 0; g < G; g++)
        if (t.p[g][j])
#pragma unroll
          for (int s = 0; s < S; s++)
#pragma unroll
            for (int e = 0; e < V; e++)
              res[g][s][e] = add_mod(res[g][s][e], mul_mod_any(x[s].v[e], pv[g].v[e], mk), mk.q);
    }
  }
#pragma unroll
  for (int g = 0; g < G; g++)
#pragma unroll
    for (int s = 0; s < S; s++) {
      if (V == 2) {
        ulonglong2 y;
        y.x = res[g][s][0];
        y.y = res[g][s][V - 1];
        *reinterpret_cast<ulonglong2*>(t.out[g] + o[s]) = y;
      } else {
        t.out[g][o[s]] = res[g][s][0];
      }
    }
}
bool launch_mul_sum_multi(const DeviceTables& T, u64* const* outs, int nouts, const u64* const* a,
                          const u64* const* p /* [nouts][nterms], null = absent */, int nterms, int nl, int bl,
                          const LimbMap& m, hipStream_t s) {
  if (nterms > SUM_MAX_TERMS || nouts > SUM_MAX_OUTS || nouts < 1 || nterms < 1) return false;
  SumMulti t;
  int present = 0;
  for (int j = 0; j < nterms; j++) t.a[j] = a[j];
  for (int g = 0; g < SUM_MAX_OUTS; g++) {
    t.out[g] = g < nouts ? outs[g] : nullptr;
    for (int j = 0; j < SUM_MAX_TERMS; j++) {
      t.p[g][j] = (g < nouts && j < nterms) ? p[(size_t)g * nterms + j] : nullptr;
      present += t.p[g][j] != nullptr;
    }
  }
  ProfScope ps("elementwise", s, 8.0 * T.N * ((double)nl * (nterms + nouts) + (double)bl * present),
               mm_map(T, m, nl, (double)T.N * present));
  int il;
  // two coefficients per thread where the ring fills whole work-groups
  const bool v2 = T.N >= (u64)(2 * TPB);
  // streams per thread: limbs bl apart share a plaintext (the map repeats
  // with a period dividing bl)
  int S = g_knobs.sum_streams;
  while (S > 1 && (bl <= 0 || nl % (bl * S) != 0 || bl % m.n != 0)) S >>= 1;
  dim3 grid = sum_grid((int)cdiv(T.N, TPB * (v2 ? 2 : 1)), nl / S, bl, g_knobs.ew_interleave, il);
  auto go = [&](auto gc, auto vc, auto sc) {
    hipLaunchKernelGGL((k_mul_sum_multi<decltype(gc)::value, decltype(vc)::value, decltype(sc)::value>), grid,
                       dim3(TPB), 0, s, t, nterms, bl, m, T.logN, T.mc, il);
  };
  auto by_s = [&](auto gc, auto vc) {
    if (S == 4) go(gc, vc, std::integral_constant<int, 4>{});
    else if (S == 2) go(gc, vc, std::integral_constant<int, 2>{});
    else go(gc, vc, std::integral_constant<int, 1>{});
  };
  auto by_v = [&](auto gc) {
    if (v2) by_s(gc, std::integral_constant<int, 2>{});
    else by_s(gc, std::integral_constant<int, 1>{});
  };
  switch (nouts) {
    case 1: by_v(std::integral_constant<int, 1>{}); break;
    case 2: by_v(std::integral_constant<int, 2>{}); break;
    case 3: by_v(std::integral_constant<int, 3>{}); break;
    default: by_v(std::integral_constant<int, 4>{}); break;
  }
  return true;
}

void launch_neg(const DeviceTables& T, u64* out, const u64* a, int nl, const LimbMap& m, hipStream_t s) {
  ew(T, EW_NEG, out, a, a, nl, nl, m, s);
}

struct ConstPairs {
  u64 w[HE_MAXMOD * 2];
};
__global__ void k_mul_const(u64* out, const u64* a, int nlimbs, ConstPairs c, LimbMap map, int logN,
                            const ModConst* __restrict__ mc) {
  const u64 N = 1ull << logN;
  u32 i = blockIdx.x * TPB + threadIdx.x;
  int k = blockIdx.y;
  if (i >= N || k >= nlimbs) return;
  int m = limb_mod(map, k);
  if (m < 0) return;
  int ci = k % map.n;
  size_t o = (size_t)k * N + i;
  out[o] = mul_const_any(a[o], c.w[2 * ci], c.w[2 * ci + 1], mc[m]);
}
void launch_mul_const(const DeviceTables& T, u64* out, const u64* a, int nlimbs, const u64* consts,
                      const LimbMap& m, hipStream_t s) {
  ConstPairs c;
  for (int k = 0; k < m.n && k < HE_MAXMOD; k++) {
    c.w[2 * k] = consts[2 * k];
    c.w[2 * k + 1] = consts[2 * k + 1];
  }
  dim3 grid(cdiv(T.N, TPB), nlimbs);
  ProfScope ps("elementwise", s, 16.0 * T.N * nlimbs, mm_map(T, m, nlimbs, (double)T.N));
  hipLaunchKernelGGL(k_mul_const, grid, dim3(TPB), 0, s, out, a, nlimbs, c, m, T.logN, T.mc);
}

// Tensor of B pairs of ciphertexts over Q_l ([2][B][nl] each):
// (a0 b0, a0 b1 + a1 b0, a1 b1) into [3][B][nl], or added onto it (ACC)
template <bool ACC>
__global__ void k_tensor(u64* out, const u64* a, const u64* b, int nl, int nt, int logN,
                         const ModConst* __restrict__ mc) {
  const u64 N = 1ull << logN;
  u32 i = blockIdx.x * TPB + threadIdx.x;
  int k = blockIdx.y;
  if (i >= N) return;
  const ModConst mk = mc[k % nl];
  size_t o0 = (size_t)k * N + i, o1 = (size_t)(nt + k) * N + i, o2 = (size_t)(2 * nt + k) * N + i;
  u64 a0 = a[o0], a1 = a[o1], b0 = b[o0], b1 = b[o1];
  if (mk.bits <= F64_LAZY_BITS) {
    // signed exact products, each output reduced once
    const double q = mk.qf, qi = mk.qinvf;
    const double x0 = u2d(a0), x1 = u2d(a1), y0 = u2d(b0), y1 = u2d(b1);
    double s0 = f64_mulmod_signed(x0, y0, q, qi);
    double s1 = f64_mulmod_signed(x0, y1, q, qi) + f64_mulmod_signed(x1, y0, q, qi);
    double s2 = f64_mulmod_signed(x1, y1, q, qi);
    if (ACC) {
      s0 += u2d(out[o0]);
      s1 += u2d(out[o1]);
      s2 += u2d(out[o2]);
    }
    out[o0] = d2u(f64_canon(s0, q, qi));
    out[o1] = d2u(f64_canon(s1, q, qi));
    out[o2] = d2u(f64_canon(s2, q, qi));
    return;
  }
  u64 t0 = mul_mod_any(a0, b0, mk);
  u64 t1 = add_mod(mul_mod_any(a0, b1, mk), mul_mod_any(a1, b0, mk), mk.q);
  u64 t2 = mul_mod_any(a1, b1, mk);
  if (ACC) {
    t0 = add_mod(t0, out[o0], mk.q);
    t1 = add_mod(t1, out[o1], mk.q);
    t2 = add_mod(t2, out[o2], mk.q);
  }
  out[o0] = t0;
  out[o1] = t1;
  out[o2] = t2;
}
// Up to TENSOR_PAIRS tensors summed in one pass, onto the running sum or not:
// each pair is read once and the three-component sum once, where one launch
// per pair reads and writes the sum for every pair.  The sum of the exact
// signed products (at most 2 TENSOR_PAIRS + 1 = 63 terms below q < 2^46
// each) stays below 2^52, so the residues are those of one pair at a time.
#define TENSOR_PAIRS 31
struct TensorPairs {
  const u64* a[TENSOR_PAIRS];
  const u64* b[TENSOR_PAIRS];
  u32 pka, pkb;  // bit p: pair p's a (b) stored packed on FP64 limbs
};
// V = 2: two consecutive coefficients per thread, 16-byte loads and stores;
// the next pair's four loads are in flight while a pair is multiplied
template <bool ACC, int V>
__global__ void __launch_bounds__(TPB) k_tensor_multi(u64* out, TensorPairs P, int npairs, int nl, int nt, int logN,
                                                      const ModConst* __restrict__ mc) {
  const u64 N = 1ull << logN;
  const u32 i = (blockIdx.x * TPB + threadIdx.x) * V;
  const int k = blockIdx.y;
  if (i >= N) return;
  const ModConst mk = mc[k % nl];
  const size_t o0 = (size_t)k * N + i, o1 = (size_t)(nt + k) * N + i, o2 = (size_t)(2 * nt + k) * N + i;
  struct W {
    u64 v[V];
  };
  auto ld = [](const u64* p) {
    W w;
    if (V == 2) {
      const ulonglong2 x = *reinterpret_cast<const ulonglong2*>(p);
      w.v[0] = x.x;
      w.v[V - 1] = x.y;
    } else {
      w.v[0] = *p;
    }
    return w;
  };
  auto st = [](u64* p, const u64 (&r)[V]) {
    if (V == 2) {
      ulonglong2 y;
      y.x = r[0];
      y.y = r[V - 1];
      *reinterpret_cast<ulonglong2*>(p) = y;
    } else {
      *p = r[0];
    }
  };
  // limb `slot` of an element at base, packed (the layout LoadPacked reads)
  // when pk: FP64 limbs of the pairs marked in P.pka / P.pkb
  const bool f64 = mk.bits <= F64_LAZY_BITS, hb1 = mk.bits <= 40;
  auto ldx = [&](const u64* base, size_t slot, bool pk) {
    if (!pk) return ld(base + slot * N + i);
    const u32* lo = reinterpret_cast<const u32*>(base + slot * N);
    W w;
    if (V == 2) {
      const uint2 l = *reinterpret_cast<const uint2*>(lo + i);
      u64 h0, h1;
      if (hb1) {
        const u32 h = *reinterpret_cast<const u16*>(reinterpret_cast<const u8*>(lo + N) + i);
        h0 = h & 255;
        h1 = h >> 8;
      } else {
        const u32 h = *reinterpret_cast<const u32*>(reinterpret_cast<const u16*>(lo + N) + i);
        h0 = h & 65535;
        h1 = h >> 16;
      }
      w.v[0] = (u64)l.x | (h0 << 32);
      w.v[V - 1] = (u64)l.y | (h1 << 32);
    } else {
      const u64 h = hb1 ? (u64) reinterpret_cast<const u8*>(lo + N)[i] : (u64) reinterpret_cast<const u16*>(lo + N)[i];
      w.v[0] = (u64)lo[i] | (h << 32);
    }
    return w;
  };
  auto pa = [&](int p) { return f64 && ((P.pka >> p) & 1u); };
  auto pb = [&](int p) { return f64 && ((P.pkb >> p) & 1u); };
  W a0n = ldx(P.a[0], k, pa(0)), a1n = ldx(P.a[0], nt + k, pa(0)), b0n = ldx(P.b[0], k, pb(0)),
    b1n = ldx(P.b[0], nt + k, pb(0));
  u64 r0[V], r1[V], r2[V];
  if (mk.bits <= F64_LAZY_BITS) {
    const double q = mk.qf, qi = mk.qinvf;
    double s0[V], s1[V], s2[V];
    if (ACC) {
      const W c0 = ld(out + o0), c1 = ld(out + o1), c2 = ld(out + o2);
#pragma unroll
      for (int e = 0; e < V; e++) {
        s0[e] = u2d(c0.v[e]);
        s1[e] = u2d(c1.v[e]);
        s2[e] = u2d(c2.v[e]);
      }
    } else {
#pragma unroll
      for (int e = 0; e < V; e++) s0[e] = s1[e] = s2[e] = 0.0;
    }
    for (int p = 0; p < npairs; p++) {
      const W a0 = a0n, a1 = a1n, b0 = b0n, b1 = b1n;
      if (p + 1 < npairs) {
        a0n = ldx(P.a[p + 1], k, pa(p + 1));
        a1n = ldx(P.a[p + 1], nt + k, pa(p + 1));
        b0n = ldx(P.b[p + 1], k, pb(p + 1));
        b1n = ldx(P.b[p + 1], nt + k, pb(p + 1));
      }
#pragma unroll
      for (int e = 0; e < V; e++) {
        const double x0 = u2d(a0.v[e]), x1 = u2d(a1.v[e]), y0 = u2d(b0.v[e]), y1 = u2d(b1.v[e]);
        s0[e] += f64_mulmod_signed(x0, y0, q, qi);
        s1[e] += f64_mulmod_signed(x0, y1, q, qi) + f64_mulmod_signed(x1, y0, q, qi);
        s2[e] += f64_mulmod_signed(x1, y1, q, qi);
      }
    }
#pragma unroll
    for (int e = 0; e < V; e++) {
      r0[e] = d2u(f64_canon(s0[e], q, qi));
      r1[e] = d2u(f64_canon(s1[e], q, qi));
      r2[e] = d2u(f64_canon(s2[e], q, qi));
    }
  } else {
    if (ACC) {
      const W c0 = ld(out + o0), c1 = ld(out + o1), c2 = ld(out + o2);
#pragma unroll
      for (int e = 0; e < V; e++) {
        r0[e] = c0.v[e];
        r1[e] = c1.v[e];
        r2[e] = c2.v[e];
      }
    } else {
#pragma unroll
      for (int e = 0; e < V; e++) r0[e] = r1[e] = r2[e] = 0;
    }
    for (int p = 0; p < npairs; p++) {
      const W a0 = a0n, a1 = a1n, b0 = b0n, b1 = b1n;
      if (p + 1 < npairs) {
        a0n = ldx(P.a[p + 1], k, pa(p + 1));
        a1n = ldx(P.a[p + 1], nt + k, pa(p + 1));
        b0n = ldx(P.b[p + 1], k, pb(p + 1));
        b1n = ldx(P.b[p + 1], nt + k, pb(p + 1));
      }
#pragma unroll
      for (int e = 0; e < V; e++) {
        r0[e] = add_mod(r0[e], mul_mod_any(a0.v[e], b0.v[e], mk), mk.q);
        r1[e] = add_mod(r1[e], add_mod(mul_mod_any(a0.v[e], b1.v[e], mk), mul_mod_any(a1.v[e], b0.v[e], mk), mk.q),
                        mk.q);
        r2[e] = add_mod(r2[e], mul_mod_any(a1.v[e], b1.v[e], mk), mk.q);
      }
    }
  }
  st(out + o0, r0);
  st(out + o1, r1);
  st(out + o2, r2);
}
void launch_tensor_sum(const DeviceTables& T, u64* out3, const u64* const* a, const u64* const* b, int npairs, int nl,
                       int batch, bool accumulate, hipStream_t s, const bool* a_packed, const bool* b_packed) {
  const int nt = nl * batch;
  // two coefficients per thread where the ring fills whole work-groups
  const bool v2 = T.N >= (u64)(2 * TPB);
  for (int p0 = 0; p0 < npairs; p0 += TENSOR_PAIRS) {
    const int np = std::min(TENSOR_PAIRS, npairs - p0);
    TensorPairs P;
    P.pka = P.pkb = 0;
    for (int p = 0; p < TENSOR_PAIRS; p++) {
      P.a[p] = p < np ? a[p0 + p] : nullptr;
      P.b[p] = p < np ? b[p0 + p] : nullptr;
      if (p < np && a_packed && a_packed[p0 + p]) P.pka |= 1u << p;
      if (p < np && b_packed && b_packed[p0 + p]) P.pkb |= 1u << p;
    }
    const bool acc = accumulate || p0 > 0;
    ProfScope ps("tensor", s, 8.0 * T.N * (4.0 * np + (acc ? 6 : 3)) * nt, mm_q(T, nl, 4.0 * T.N * np, batch));
    dim3 grid(cdiv(T.N, TPB * (v2 ? 2 : 1)), nt);
    if (acc && v2) hipLaunchKernelGGL((k_tensor_multi<true, 2>), grid, dim3(TPB), 0, s, out3, P, np, nl, nt, T.logN, T.mc);
    else if (acc) hipLaunchKernelGGL((k_tensor_multi<true, 1>), grid, dim3(TPB), 0, s, out3, P, np, nl, nt, T.logN, T.mc);
    else if (v2) hipLaunchKernelGGL((k_tensor_multi<false, 2>), grid, dim3(TPB), 0, s, out3, P, np, nl, nt, T.logN, T.mc);
    else hipLaunchKernelGGL((k_tensor_multi<false, 1>), grid, dim3(TPB), 0, s, out3, P, np, nl, nt, T.logN, T.mc);
  }
}

void launch_tensor(const DeviceTables& T, u64* out3, const u64* a, const u64* b, int nl, int batch, bool accumulate,
                   hipStream_t s) {
  const int nt = nl * batch;
  ProfScope ps("tensor", s, 8.0 * T.N * (accumulate ? 10 : 7) * nt, mm_q(T, nl, 4.0 * T.N, batch));
  dim3 grid(cdiv(T.N, TPB), nt);
  if (accumulate) hipLaunchKernelGGL(k_tensor<true>, grid, dim3(TPB), 0, s, out3, a, b, nl, nt, T.logN, T.mc);
  else hipLaunchKernelGGL(k_tensor<false>, grid, dim3(TPB), 0, s, out3, a, b, nl, nt, T.logN, T.mc);
}

__global__ void k_int_to_limbs(u64* out, const i64* in, int nlimbs, LimbMap map, int logN,
                               const ModConst* __restrict__ mc) {
  const u64 N = 1ull << logN;
  u32 i = blockIdx.x * TPB + threadIdx.x;
  int k = blockIdx.y;
  if (i >= N) return;
  int m = limb_mod(map, k);
  if (m < 0) return;
  out[(size_t)k * N + i] = reduce_signed(in[i], mc[m]);
}
void launch_int_to_limbs(const DeviceTables& T, u64* out, const i64* in, int nlimbs, const LimbMap& m,
                         hipStream_t s) {
  dim3 grid(cdiv(T.N, TPB), nlimbs);
  hipLaunchKernelGGL(k_int_to_limbs, grid, dim3(TPB), 0, s, out, in, nlimbs, m, T.logN, T.mc);
}

// ---------------------------------------------------------------------------
// Key switching: Decompose (ModUp), MultSum, ModDown
// ---------------------------------------------------------------------------
struct ModupArgs {
  int nq, nqp, alpha, beta, L;
  int ns[16];
  u64 hatinv[16][4], hatinv_sh[16][4];
  const u64* hat_t[16];
  const u64* hat_t_sh[16];
};

// digits[j][pos][i]: coefficient-domain fast basis conversion of digit j to
// every modulus of Q_l and P; the digit's own limbs receive the input itself.
__global__ void k_modup(u64* digits, const u64* coef, const u64* ntt_in, ModupArgs A, int logN, int nmods,
                        const ModConst* __restrict__ mc) {
  const u64 N = 1ull << logN;
  u32 i = blockIdx.x * TPB + threadIdx.x;
  int j = blockIdx.y;
  // batch member blockIdx.z: inputs [B][nq][N], digits [B][beta][nqp][N]
  digits += (size_t)blockIdx.z * A.beta * A.nqp * N;
  coef += (size_t)blockIdx.z * A.nq * N;
  ntt_in += (size_t)blockIdx.z * A.nq * N;
  const int ns = A.ns[j];
  // the digit's conversion constants (ns x nmods, with Shoup companions) staged in LDS
  __shared__ u64 hat_l[4 * HE_MAXMOD], hat_sh_l[4 * HE_MAXMOD];
  for (int e = threadIdx.x; e < ns * nmods; e += TPB) {
    hat_l[e] = A.hat_t[j][e];
    hat_sh_l[e] = A.hat_t_sh[j][e];
  }
  __syncthreads();
  if (i >= N) return;
  u64 y[4];
  u32 src_bits = 0;
  for (int a = 0; a < ns; a++) {
    int sm = j * A.alpha + a;
    u64 x = coef[(size_t)sm * N + i];
    y[a] = mul_const_any(x, A.hatinv[j][a], A.hatinv_sh[j][a], mc[sm]);
    src_bits = max(src_bits, mc[sm].bits);
  }
  for (int pos = 0; pos < A.nqp; pos++) {
    u64* o = digits + ((size_t)j * A.nqp + pos) * N + i;
    if (pos < A.nq && pos / A.alpha == j) {
      *o = ntt_in[(size_t)pos * N + i];
      continue;
    }
    int m = pos < A.nq ? pos : A.L + 1 + (pos - A.nq);
    const ModConst& mt = mc[m];
    const u64* hat = hat_l + m;
    const u64* hat_sh = hat_sh_l + m;
    if (mt.bits <= F64_LAZY_BITS && src_bits <= mt.bits + 1) {
      // inputs below 4 q_t: signed exact products, summed, reduced once
      double acc = 0.0;
      for (int a = 0; a < ns; a++) acc += f64_mulmod_signed(u2d(y[a]), u2d(hat[(size_t)a * nmods]), mt.qf, mt.qinvf);
      *o = d2u(f64_canon(acc, mt.qf, mt.qinvf));
    } else {
      u64 acc = 0;
      for (int a = 0; a < ns; a++)
        acc = add_mod(acc, shoup_mul(y[a], hat[(size_t)a * nmods], hat_sh[(size_t)a * nmods], mt.q), mt.q);
      *o = acc;
    }
  }
}

void launch_modup(const DeviceTables& T, u64* digits, const u64* coef, const u64* ntt_in, int level, int L,
                  int alpha, int beta, const FbcTable* tabs, int batch, hipStream_t s) {
  ModupArgs A;
  A.nq = level + 1;
  A.nqp = level + 1 + alpha;
  A.alpha = alpha;
  A.beta = beta;
  A.L = L;
  for (int j = 0; j < beta; j++) {
    A.ns[j] = tabs[j].ns;
    for (int a = 0; a < tabs[j].ns; a++) {
      A.hatinv[j][a] = tabs[j].hatinv[a];
      A.hatinv_sh[j][a] = tabs[j].hatinv_sh[a];
    }
    A.hat_t[j] = tabs[j].hat_t;
    A.hat_t_sh[j] = tabs[j].hat_t_sh;
  }
  Mm mm;
  for (int j = 0; j < beta; j++)
    mm = mm + mm_qp(T, level + 1, level + 1 + alpha, L, (double)T.N * tabs[j].ns, (double)T.N * tabs[j].ns, batch);
  mm = mm + mm_q(T, level + 1, (double)T.N, batch);
  ProfScope ps("modup", s, 8.0 * T.N * batch * ((level + 1) + (double)beta * (level + 1 + alpha)), mm);
  dim3 grid(cdiv(T.N, TPB), beta, batch);
  hipLaunchKernelGGL(k_modup, grid, dim3(TPB), 0, s, digits, coef, ntt_in, A, T.logN, T.nmods, T.mc);
}

struct FbcArgs {
  int ns;
  int src[4];
  u64 hatinv[4], hatinv_sh[4];
  const u64* hat_t;
  const u64* hat_t_sh;
  u64 Dw[4];
  u64 Hw[4][4];
  double qrecip[4];   // 1 / q_a of the sources
  const u64* D_mod_t;
  const double* hat_f;
  int src_stride, src_off;  // source limb a of poly p at slot p * src_stride + src_off + a
};

// acc (4 words) += H (4 words) * y, carries beyond the top word dropped
__device__ __forceinline__ void w4_muladd(u64 acc[4], const u64 H[4], u64 y) {
  u64 carry = 0;
#pragma unroll
  for (int k = 0; k < 4; k++) {
    u64 lo = H[k] * y, hi = mulhi64(H[k], y);
    u64 s = acc[k] + lo;
    u64 c1 = s < lo;
    u64 s2 = s + carry;
    u64 c2 = s2 < carry;
    acc[k] = s2;
    carry = hi + c1 + c2;
  }
}
__device__ __forceinline__ int w4_cmp(const u64 a[4], const u64 b[4]) {
  for (int k = 3; k >= 0; k--)
    if (a[k] != b[k]) return a[k] < b[k] ? -1 : 1;
  return 0;
}

// round(S / D) for S = sum_a y_a (D / q_a), 0 <= y_a < q_a: a double estimate
// of sum_a y_a / q_a (products with the rounded reciprocals: error below
// ns 2^-52), replaced by an exact multiword comparison when the estimate lies
// within 2^-40 of a rounding boundary.
__device__ __forceinline__ u64 round_quotient(const u64* y, const FbcArgs& A) {
  double f = 0.0;
  for (int a = 0; a < A.ns; a++) f += (double)y[a] * A.qrecip[a];
  double t = f + 0.5;
  double fl = floor(t);
  double fr = t - fl;
  if (fr > 9.094947017729282e-13 && fr < 1.0 - 9.094947017729282e-13) return (u64)fl;
  // exact: v = #{ w >= 1 : 2 S > (2w - 1) D }
  u64 S2[4] = {0, 0, 0, 0};
  for (int a = 0; a < A.ns; a++) w4_muladd(S2, A.Hw[a], 2 * y[a]);
  u64 v = 0;
  for (u64 w = 1; w <= (u64)A.ns; w++) {
    u64 T[4] = {0, 0, 0, 0};
    w4_muladd(T, A.Dw, 2 * w - 1);
    if (w4_cmp(S2, T) > 0) v = w;
  }
  return v;
}

// y[t][i] = ([x]_D mod q_t) for t < nq, with [x]_D the exact centred residue
// of the source limbs x (coefficient domain); batch over polys (grid.z)
__global__ void k_fbc_to_q(u64* y, const u64* xp, int nq, FbcArgs A, int logN, int nmods,
                           const ModConst* __restrict__ mc) {
  const u64 N = 1ull << logN;
  u32 i = blockIdx.x * TPB + threadIdx.x;
  if (i >= N) return;
  int poly = blockIdx.z;
  const u64* x = xp + (size_t)poly * A.ns * N;
  u64* yy = y + (size_t)poly * nq * N;
  u64 v[4];
  for (int a = 0; a < A.ns; a++) v[a] = shoup_mul(x[(size_t)a * N + i], A.hatinv[a], A.hatinv_sh[a], mc[A.src[a]].q);
  const u64 r = round_quotient(v, A);
  for (int t = blockIdx.y; t < nq; t += gridDim.y) {
    const ModConst& mt = mc[t];
    if (mt.bits <= F64_LAZY_BITS && mt.bits > 32) {
      // v = v_hi 2^32 + v_lo with both halves below q_t: exact signed FP64
      // products, summed, reduced once
      const double q = mt.qf, qi = mt.qinvf;
      double acc = 0.0;
      for (int a = 0; a < A.ns; a++) {
        const double* e = A.hat_f + ((size_t)a * nmods + t) * 3;
        acc += f64_mulmod_signed(u2d(v[a] & 0xffffffffull), e[0], q, qi);
        acc += f64_mulmod_signed(u2d(v[a] >> 32), e[1], q, qi);
      }
      acc -= f64_mulmod_signed(u2d(r), A.hat_f[(size_t)t * 3 + 2], q, qi);
      yy[(size_t)t * N + i] = d2u(f64_canon(acc, q, qi));
    } else {
      u64 q = mt.q, acc = 0;
      for (int a = 0; a < A.ns; a++)
        acc = add_mod(acc, shoup_mul(v[a], A.hat_t[(size_t)a * nmods + t], A.hat_t_sh[(size_t)a * nmods + t], q), q);
      acc = sub_mod(acc, shoup_mul(r, A.D_mod_t[2 * t], A.D_mod_t[2 * t + 1], q), q);
      yy[(size_t)t * N + i] = acc;
    }
  }
}
void launch_fbc_to_q(const DeviceTables& T, u64* y, const u64* xp_coef, int nq, int npoly, const FbcTable& tab,
                     hipStream_t s) {
  FbcArgs A;
  A.ns = tab.ns;
  for (int a = 0; a < tab.ns; a++) {
    A.src[a] = tab.src[a];
    A.hatinv[a] = tab.hatinv[a];
    A.hatinv_sh[a] = tab.hatinv_sh[a];
    A.qrecip[a] = 1.0 / tab.qd[a];
    for (int w = 0; w < 4; w++) A.Hw[a][w] = tab.Hw[a][w];
  }
  for (int w = 0; w < 4; w++) A.Dw[w] = tab.Dw[w];
  A.hat_t = tab.hat_t;
  A.hat_t_sh = tab.hat_t_sh;
  A.D_mod_t = tab.D_mod_t;
  A.hat_f = tab.hat_f;
  A.src_stride = tab.ns;
  A.src_off = 0;
  ProfScope ps("fbc_to_q", s, 8.0 * T.N * npoly * ((double)tab.ns + nq), mm_q(T, nq, (double)T.N * (tab.ns + 1), npoly));
  dim3 grid(cdiv(T.N, TPB), nq < 4 ? nq : 4, npoly);
  hipLaunchKernelGGL(k_fbc_to_q, grid, dim3(TPB), 0, s, y, xp_coef, nq, A, T.logN, T.nmods, T.mc);
}

// ModDown with the basis conversion fused into the forward column pass.
// k_fbc_prep stores, per coefficient, v_a = x_a hatinv_a mod p_a and the
// rounded quotient r of the exact centred lift ([npoly][ns + 1][N]); the
// column pass of target limb t then loads
//   sum_a v_a hat_(a,t) - r D mod q_t
// (the value k_fbc_to_q writes) while filling its tile, and the block pass
// ends with (x - y) P^-1: no converted limb goes to memory.
__global__ void k_fbc_prep(u64* V, const u64* xp, FbcArgs A, int logN, const ModConst* __restrict__ mc) {
  const u64 N = 1ull << logN;
  u32 i = blockIdx.x * TPB + threadIdx.x;
  if (i >= N) return;
  const int poly = blockIdx.y;
  const u64* x = xp + ((size_t)poly * A.src_stride + A.src_off) * N;
  u64* o = V + (size_t)poly * (A.ns + 1) * N;
  u64 v[4];
  for (int a = 0; a < A.ns; a++) v[a] = shoup_mul(x[(size_t)a * N + i], A.hatinv[a], A.hatinv_sh[a], mc[A.src[a]].q);
  const u64 r = round_quotient(v, A);
  for (int a = 0; a < A.ns; a++) o[(size_t)a * N + i] = v[a];
  o[(size_t)A.ns * N + i] = r;
}
// F64 (target of 33 to 46 bits): v = v_hi 2^32 + v_lo, both halves below
// q_t, signed exact products, one reduction; otherwise Shoup products.  No
// branches on the source count: NS = 3 for three special primes, else 4 with
// sources past ns repeating the last one against zero constants.
struct FbcData {
  const u64* v0;
  u64 N;
  int ns;
  u64 q, h[4], hs[4], D, Ds;
  double qf, qinvf, e0[4], e1[4], e2;
};
template <bool F64, int NS = 4>
struct FbcLoad : FbcData {
  struct Raw {
    u64 x[NS], r;
  };
  __device__ __forceinline__ void raw(size_t idx, Raw& w) const {
#pragma unroll
    for (int a = 0; a < NS; a++) w.x[a] = v0[(size_t)(a < ns ? a : ns - 1) * N + idx];
    w.r = v0[(size_t)ns * N + idx];
  }
  __device__ __forceinline__ double sum_f64(const Raw& w) const {
    // the quotient r is at most the source count: r D is exact (below 2^49)
    double acc = -u2d(w.r) * e2;
#pragma unroll
    for (int a = 0; a < NS; a++) {
      acc += f64_mulmod_signed(u2d(w.x[a] & 0xffffffffull), e0[a], qf, qinvf);
      acc += f64_mulmod_signed(u2d(w.x[a] >> 32), e1[a], qf, qinvf);
    }
    return acc;
  }
  __device__ __forceinline__ u64 fin_u(const Raw& w) const {
    if (F64) return d2u(f64_canon(sum_f64(w), qf, qinvf));
    u64 acc = 0;
#pragma unroll
    for (int a = 0; a < NS; a++) acc = add_mod(acc, shoup_mul(w.x[a], h[a], hs[a], q), q);
    return sub_mod(acc, shoup_mul(w.r, D, Ds, q), q);
  }
  __device__ __forceinline__ double fin_d(const Raw& w) const { return f64_centre(sum_f64(w), qf, qinvf); }
};
template <int NS>
__device__ __forceinline__ double fin(const F64LazyArith&, const FbcLoad<true, NS>& ld,
                                      const typename FbcLoad<true, NS>::Raw& w) {
  return ld.fin_d(w);
}
template <class L>
__device__ __forceinline__ L fbc_loader_of(const FbcData& d) {
  L l;
  static_cast<FbcData&>(l) = d;
  return l;
}
template <int LOGN, int GA, int GB>
__global__ void __launch_bounds__(TPB) k_ntt_cols2_fbc(u64* y, const u64* __restrict__ V, int nq, FbcArgs A,
                                                       const u64* __restrict__ tw, const u64* __restrict__ twsh,
                                                       const double* __restrict__ twf, int nmods,
                                                       const ModConst* __restrict__ mc) {
  constexpr int S1 = GA + GB, R = 1 << S1, C = TILE / R;
  __shared__ u64 sh[LDS_WORDS];
  const int limb = blockIdx.y;
  const int p = limb / nq, t = limb - p * nq;
  const u64 N = 1ull << LOGN;
  u64* a = y + (size_t)limb * N;
  const int c0 = blockIdx.x * C;
  const ModConst mk = mc[t];
  FbcData d;
  d.v0 = V + (size_t)p * (A.ns + 1) * N;
  d.N = N;
  d.ns = A.ns;
  d.q = mk.q;
  d.qf = mk.qf;
  d.qinvf = mk.qinvf;
  d.D = A.D_mod_t[2 * t];
  d.Ds = A.D_mod_t[2 * t + 1];
  d.e2 = A.hat_f[(size_t)t * 3 + 2];
  for (int x = 0; x < 4; x++) {
    const bool in = x < A.ns;
    d.h[x] = in ? A.hat_t[(size_t)x * nmods + t] : 0;
    d.hs[x] = in ? A.hat_t_sh[(size_t)x * nmods + t] : 0;
    d.e0[x] = in ? A.hat_f[((size_t)x * nmods + t) * 3] : 0.0;
    d.e1[x] = in ? A.hat_f[((size_t)x * nmods + t) * 3 + 1] : 0.0;
  }
  if (mk.bits <= F64_LAZY_BITS) {
    F64LazyArith ar{twf + (size_t)t * N, mk.qf, mk.qinvf, (double)mk.ninv};
    double* shd = reinterpret_cast<double*>(sh);
    if (mk.bits <= 32)
      ntt_cols2_body<LOGN, GA, GB, false>(a, c0, shd, ar, fbc_loader_of<FbcLoad<false>>(d));
    else if (d.ns == 3)  // three special primes: no padding source
      ntt_cols2_body<LOGN, GA, GB, false>(a, c0, shd, ar, fbc_loader_of<FbcLoad<true, 3>>(d));
    else
      ntt_cols2_body<LOGN, GA, GB, false>(a, c0, shd, ar, fbc_loader_of<FbcLoad<true>>(d));
  } else {
    ShoupArith ar{tw + (size_t)t * N, twsh + (size_t)t * N, mk.q, mk.ninv, mk.ninv_sh};
    ntt_cols2_body<LOGN, GA, GB, false>(a, c0, sh, ar, fbc_loader_of<FbcLoad<false>>(d));
  }
}
// ModDown's lift as an int8 matrix product.  k_fbc_prep_digits writes, per
// coefficient, a record of kw words: byte 9 a + i is 7-bit digit i of the
// source value v_a (nine digits cover 63 bits), byte 9 ns the rounded
// quotient r, the rest zero.  For a target t the lift
//   sum_a v_a hat_(a,t) - r D  =  sum_k x_k C_(k,t)    (mod q_t)
// with x_k the record bytes and C_(k,t) = hat_(a,t) 2^(7 i) mod q_t (-D mod
// q_t for the quotient); cutting each constant into seven 7-bit digits,
//   S_j = sum_k x_k digit_j(C_(k,t))  < 37 * 127 * 127 < 2^19.2
// is a dot product of bytes, and the lift is sum_j S_j 2^(7 j) mod q_t.
struct FbcTgts {
  short t[64];
  int n;
};
// Work-groups are dispatched to the 8 XCDs in turn (work-group b to XCD
// b % 8), and each XCD has its own L2.  xcd_perm renumbers the first
// 8 * floor(n / 8) of n work-groups so that XCD x runs the x-th contiguous
// range of logical work-groups (launch order kept within it): work-groups
// that read the same data (the tiles of one polynomial) share an L2.  The
// rest keep their numbers.
__device__ __forceinline__ int xcd_perm(int b, int n) {
  const int per = n >> 3;
  return b < per * 8 ? (b & 7) * per + (b >> 3) : b;
}
// KB record bytes, KU stored words, KW words the products read (whole
// 16-byte steps: the words past KU are zero and not stored)
template <int NS>
struct FbcRec {
  static constexpr int KB = 9 * NS + 1, KU = (KB + 7) / 8, KW = 2 * ((KB + 15) / 16);
  static_assert(KU == NS + 1, "a record takes the words of the sources and the quotient");
};
template <int NS>
__global__ void k_fbc_prep_digits(u64* V, const u64* xp, FbcArgs A, int logN, const ModConst* __restrict__ mc) {
  constexpr int KU = FbcRec<NS>::KU;
  const u64 N = 1ull << logN;
  u32 i = blockIdx.x * TPB + threadIdx.x;
  if (i >= N) return;
  const int poly = blockIdx.y;
  const u64* x = xp + ((size_t)poly * A.src_stride + A.src_off) * N;
  u64* o = V + (size_t)poly * KU * N;
  u64 v[4];
#pragma unroll
  for (int a = 0; a < NS; a++) v[a] = shoup_mul(x[(size_t)a * N + i], A.hatinv[a], A.hatinv_sh[a], mc[A.src[a]].q);
  const u64 r = round_quotient(v, A);
  u64 w[KU];
#pragma unroll
  for (int k = 0; k < KU; k++) w[k] = 0;
#pragma unroll
  for (int a = 0; a < NS; a++)
#pragma unroll
    for (int d = 0; d < 9; d++) {
      const int k = 9 * a + d;
      w[k >> 3] |= ((v[a] >> (7 * d)) & 127) << (8 * (k & 7));
    }
  w[(9 * NS) >> 3] |= r << (8 * ((9 * NS) & 7));
#pragma unroll
  for (int k = 0; k < KU; k++) o[(size_t)k * N + i] = w[k];
}

// The column pass of targets outside the FP64 path (and any target) from the
// record: the source values are reassembled from their digits, then the
// Shoup lift of FbcLoad<false>.
template <int NS>
struct FbcDigitLoad {
  static constexpr int KU = FbcRec<NS>::KU;
  struct Raw {
    u64 w[KU];
  };
  const u64* v0;
  u64 N;
  u64 q, h[4], hs[4], D, Ds;
  __device__ __forceinline__ void raw(size_t idx, Raw& r) const {
#pragma unroll
    for (int k = 0; k < KU; k++) r.w[k] = v0[(size_t)k * N + idx];
  }
  __device__ __forceinline__ static u64 byte(const Raw& r, int k) { return (r.w[k >> 3] >> (8 * (k & 7))) & 255; }
  __device__ __forceinline__ u64 fin_u(const Raw& r) const {
    u64 acc = 0;
#pragma unroll
    for (int a = 0; a < NS; a++) {
      u64 v = 0;
#pragma unroll
      for (int d = 0; d < 9; d++) v |= byte(r, 9 * a + d) << (7 * d);
      acc = add_mod(acc, shoup_mul(v, h[a], hs[a], q), q);
    }
    return sub_mod(acc, shoup_mul(byte(r, 9 * NS), D, Ds, q), q);
  }
};
// The inverse column pass of the ns ModDown sources of one polynomial (one
// TPB-thread group per source limb, every barrier outside the arithmetic's
// branches), finished into the digit records k_fbc_prep_digits writes: the
// coefficient values stay in LDS and only the records go to memory, rec
// [polynomial][ns + 1][N] in the order of the launch's element table.
template <int LOGN, int GA, int GB, class A>
__device__ __forceinline__ void intt_cols_first(const u64* a, int c0, typename A::V* sh, const A& ar, int tid) {
  typedef typename A::V V;
  constexpr int S1 = GA + GB, R = 1 << S1, T1 = (1 << LOGN) / R, C = TILE / R, S2 = LOGN - S1, ITB = 16 >> GB;
  V v[16];
#pragma unroll
  for (int k = 0; k < ITB; k++) {
    const int it = tid + TPB * k, c = it % C, rh = it / C;
#pragma unroll
    for (int mm = 0; mm < (1 << GB); mm++) v[mm] = ar.load(a[(size_t)((rh << GB) + mm) * T1 + c0 + c]);
    inv_group<GB>(v, S2, LOGN, (u32)rh, ar);
#pragma unroll
    for (int mm = 0; mm < (1 << GB); mm++) sh[lds_rc((rh << GB) + mm, c, C)] = v[mm];
  }
}
template <int LOGN, int GA, int GB, class A>
__device__ __forceinline__ void intt_cols_last_lds(typename A::V* sh, const A& ar, int tid) {
  typedef typename A::V V;
  constexpr int S1 = GA + GB, R = 1 << S1, C = TILE / R, S2 = LOGN - S1, ITA = 16 >> GA;
  V v[16];
#pragma unroll
  for (int k = 0; k < ITA; k++) {
    const int it = tid + TPB * k, c = it % C, rl = it / C;
#pragma unroll
    for (int mm = 0; mm < (1 << GA); mm++) v[mm] = ar.reduce(sh[lds_rc(rl + (mm << GB), c, C)]);
    inv_group_last_scaled<GA>(v, S2 + GB, LOGN, ar);
    // canonical residues, in place (positions only this thread reads)
#pragma unroll
    for (int mm = 0; mm < (1 << GA); mm++)
      reinterpret_cast<u64*>(sh)[lds_rc(rl + (mm << GB), c, C)] = ar.store(v[mm]);
  }
}
template <int LOGN, int GA, int GB, int NS>
__global__ void __launch_bounds__(NS * TPB)
    k_intt_cols2_rec(LimbBases lb, LimbMap map, FbcArgs A, u64* rec, const u64* __restrict__ tw,
                     const u64* __restrict__ twsh, const double* __restrict__ twf, const ModConst* __restrict__ mc) {
  constexpr int S1 = GA + GB, R = 1 << S1, T1 = (1 << LOGN) / R, C = TILE / R, KU = FbcRec<NS>::KU;
  __shared__ u64 sh[NS][LDS_WORDS];
  const int src = threadIdx.x / TPB, tid = threadIdx.x - src * TPB;
  const int poly = blockIdx.y;
  const u64 N = 1ull << LOGN;
  const u64* a = limb_base_addr(lb, poly * NS + src, N);
  const int c0 = blockIdx.x * C;
  const ModConst mk = mc[map.idx[src]];
  const int m = map.idx[src];
  const bool f64 = mk.bits <= F64_LAZY_BITS;
  const F64LazyArith af{twf + (size_t)m * N, mk.qf, mk.qinvf, (double)mk.ninv};
  const ShoupArith as{tw + (size_t)m * N, twsh + (size_t)m * N, mk.q, mk.ninv, mk.ninv_sh};
  if (f64) intt_cols_first<LOGN, GA, GB>(a, c0, reinterpret_cast<double*>(sh[src]), af, tid);
  else intt_cols_first<LOGN, GA, GB>(a, c0, sh[src], as, tid);
  __syncthreads();
  if (f64) intt_cols_last_lds<LOGN, GA, GB>(reinterpret_cast<double*>(sh[src]), af, tid);
  else intt_cols_last_lds<LOGN, GA, GB>(sh[src], as, tid);
  __syncthreads();
  u64* o = rec + (size_t)poly * KU * N;
  for (int e = threadIdx.x; e < TILE; e += NS * TPB) {
    const int row = e / C, col = e % C;
    u64 v[4];
#pragma unroll
    for (int x = 0; x < NS; x++)
      v[x] = shoup_mul(sh[x][lds_rc(row, col, C)], A.hatinv[x], A.hatinv_sh[x], mc[A.src[x]].q);
    const u64 r = round_quotient(v, A);
    u64 w[KU];
#pragma unroll
    for (int k = 0; k < KU; k++) w[k] = 0;
#pragma unroll
    for (int x = 0; x < NS; x++)
#pragma unroll
      for (int d = 0; d < 9; d++) {
        const int k = 9 * x + d;
        w[k >> 3] |= ((v[x] >> (7 * d)) & 127) << (8 * (k & 7));
      }
    w[(9 * NS) >> 3] |= r << (8 * ((9 * NS) & 7));
    const size_t i = (size_t)row * T1 + c0 + col;
#pragma unroll
    for (int k = 0; k < KU; k++) o[(size_t)k * N + i] = w[k];
  }
}

template <int LOGN, int GA, int GB, int GC, int GD>
static void intt2_many(const DeviceTables& T, const LimbBases& lb, int nelem, const LimbMap& map, hipStream_t s,
                       const FbcArgs* fa, u64* rec) {
  constexpr int R = 1 << (GA + GB), C = TILE / R, T1 = 1 << (GC + GD), K = TILE / T1;
  const int nlimbs = nelem * lb.per_elem;
  dim3 gc((1 << LOGN) / R / C, nlimbs), gr(((1 << LOGN) / T1) / K, nlimbs);
  // the modulus pattern repeats every `per` limbs, and per_elem is a multiple of it
  const int il = interleave_of(nlimbs, modulus_period(map), g_knobs.ntt_interleave);
  const double pass_bytes = 16.0 * nlimbs * T.N;
  {
    ProfScope ps("ntt_inv_rows", s, pass_bytes, mm_map(T, map, nlimbs, 0.5 * T.N * (GC + GD)));
    hipLaunchKernelGGL((k_intt_rows2_many<LOGN, GC, GD>), gr, dim3(TPB), 0, s, lb, map, T.ipsi, T.ipsi_sh, T.ipsi_f,
                       T.mc, il);
  }
  if (!rec) {
    ProfScope ps("ntt_inv_cols", s, pass_bytes, mm_map(T, map, nlimbs, 0.5 * T.N * (GA + GB)));
    hipLaunchKernelGGL((k_intt_cols2_many<LOGN, GA, GB>), gc, dim3(TPB), 0, s, lb, map, T.ipsi, T.ipsi_sh, T.ipsi_f,
                       T.mc);
    return;
  }
  // the last pass ends in the digit records: the sources are read once and
  // only the records ((ns + 1) words a coefficient) are written
  const int npoly = nlimbs / lb.per;
  Mm mm = mm_map(T, map, nlimbs, 0.5 * T.N * (GA + GB));
  for (int a = 0; a < fa->ns; a++) mm.add(T.bits[fa->src[a]], (double)T.N * npoly);
  ProfScope ps("ntt_inv_cols", s, 8.0 * T.N * (nlimbs + (double)npoly * (fa->ns + 1)), mm);
  dim3 g((1 << LOGN) / R / C, npoly);
  switch (lb.per) {
    case 1: hipLaunchKernelGGL((k_intt_cols2_rec<LOGN, GA, GB, 1>), g, dim3(1 * TPB), 0, s, lb, map, *fa, rec, T.ipsi, T.ipsi_sh, T.ipsi_f, T.mc); break;
    case 2: hipLaunchKernelGGL((k_intt_cols2_rec<LOGN, GA, GB, 2>), g, dim3(2 * TPB), 0, s, lb, map, *fa, rec, T.ipsi, T.ipsi_sh, T.ipsi_f, T.mc); break;
    case 3: hipLaunchKernelGGL((k_intt_cols2_rec<LOGN, GA, GB, 3>), g, dim3(3 * TPB), 0, s, lb, map, *fa, rec, T.ipsi, T.ipsi_sh, T.ipsi_f, T.mc); break;
    default: hipLaunchKernelGGL((k_intt_cols2_rec<LOGN, GA, GB, 4>), g, dim3(4 * TPB), 0, s, lb, map, *fa, rec, T.ipsi, T.ipsi_sh, T.ipsi_f, T.mc); break;
  }
}

static FbcArgs fbc_args(const FbcTable& tab, int src_stride, int src_off);
void launch_intt_many(const DeviceTables& T, const std::vector<u64*>& bases, int per_elem, int per, int stride,
                      int off, const LimbMap& map, hipStream_t s, const FbcTable* rec_tab, u64* rec) {
  if (map.n != per || per_elem % per != 0) throw std::runtime_error("launch_intt_many: bad limb pattern");
  if (rec && (!rec_tab || rec_tab->ns != per || per > 4))
    throw std::runtime_error("launch_intt_many: records need the ModDown table of the sources");
  FbcArgs fa;
  if (rec) fa = fbc_args(*rec_tab, per, 0);
  for (size_t e0 = 0; e0 < bases.size(); e0 += MR_MAX) {
    const int ne = (int)std::min(bases.size() - e0, (size_t)MR_MAX);
    LimbBases lb;
    for (int e = 0; e < MR_MAX; e++) lb.base[e] = e < ne ? bases[e0 + e] : nullptr;
    lb.per_elem = per_elem;
    lb.per = per;
    lb.stride = stride;
    lb.off = off;
    u64* rc = rec ? rec + (size_t)e0 * (per_elem / per) * (per + 1) * T.N : nullptr;
    if (!ntt_dispatch(T.logN, [&](auto sp) {
          using S = decltype(sp);
          intt2_many<NTT_SPLIT_ARGS>(T, lb, ne, map, s, rec ? &fa : nullptr, rc);
        }))
      throw std::runtime_error("launch_intt_many needs the register-blocked NTT (log N 12..16)");
  }
}

typedef int mfma_i32x16 __attribute__((ext_vector_type(16)));
// Two FP64 targets (33 to 46 bits) t0, t1 per work-group of 2 TPB threads.
// v_mfma_i32_32x32x16_i8 takes, per lane l:
//   A (32 x 16) row i = l % 32, bytes k = 8 (l / 32) + 0..7: rows 0-3 and
//     8-11 hold digits 0-3 and 4-7 of t0's constants, rows 4-7 and 12-15
//     those of t1 (row 7 of each is zero), rows 16-31 zero;
//   B (16 x 32) column l % 32: the same bytes of a coefficient's record;
//   D row 8 (r / 4) + 4 (l / 32) + r % 4, column l % 32,
// so that register r < 7 of lane l is S_r of target t_(l / 32) for the
// coefficient of column l % 32.  Lane i < 32 of wave w (both halves) takes
// as its columns the values the column pass's thread 32 w + i loads (16 per
// thread), and so ends holding that thread's values for target t_(l / 32):
// the first stage group runs in registers, the second from the LDS tile of
// the lane's target.
// The launch's first work-groups (blockIdx.y below ceil(to.n npoly / 2))
// instead run the targets of the Shoup path (above 46 bits, q0): two
// (polynomial, target) units each, one per half, from the same records.
template <int LOGN, int GA, int GB, int NS>
__global__ void __launch_bounds__(2 * TPB) __attribute__((amdgpu_waves_per_eu(4)))
    k_ntt_cols2_fbc_mfma(u64* y, const u64* __restrict__ V, int nq, int npoly, FbcTgts tg, FbcTgts to, FbcArgs A,
                         const u64* __restrict__ cdig, const u64* __restrict__ tw, const u64* __restrict__ twsh,
                         const double* __restrict__ twf, int nmods, const ModConst* __restrict__ mc, int xcd_map) {
  constexpr int S1 = GA + GB, R = 1 << S1, T1 = (1 << LOGN) / R, C = TILE / R, KW = FbcRec<NS>::KW,
                KU = FbcRec<NS>::KU;
  constexpr int ITA = 16 >> GA, NA = 1 << GA, ITB = 16 >> GB;
  __shared__ double sh[2][LDS_WORDS];
  // the Shoup-path work-groups first, in launch order (spread over the
  // XCDs); the MFMA ones after them, grouped by XCD when xcd_map is set
  const int gx = gridDim.x, nint = (to.n * npoly + 1) >> 1;
  int b = blockIdx.y * gx + blockIdx.x;
  if (xcd_map && b >= nint * gx) b = nint * gx + xcd_perm(b - nint * gx, gx * (gridDim.y - nint));
  int by = b / gx;
  const int bx = b - by * gx;
  const u64 N = 1ull << LOGN;
  const int c0 = bx * C;
  if (by < nint) {
    const int hs = threadIdx.x >= TPB, tid = threadIdx.x - hs * TPB;
    int u = 2 * by + hs;
    const bool act = u < to.n * npoly;
    if (!act) u = 2 * by;  // an odd unit count: this half computes and stores nothing
    const int p = u / to.n, t = to.t[u - p * to.n];
    const ModConst mk = mc[t];
    FbcDigitLoad<NS> ld;
    ld.v0 = V + (size_t)p * KU * N;
    ld.N = N;
    ld.q = mk.q;
    ld.D = A.D_mod_t[2 * t];
    ld.Ds = A.D_mod_t[2 * t + 1];
#pragma unroll
    for (int x = 0; x < NS; x++) {
      ld.h[x] = A.hat_t[(size_t)x * nmods + t];
      ld.hs[x] = A.hat_t_sh[(size_t)x * nmods + t];
    }
    ShoupArith ar{tw + (size_t)t * N, twsh + (size_t)t * N, mk.q, mk.ninv, mk.ninv_sh};
    ntt_cols2_fwd<LOGN, GA, GB>(y + ((size_t)p * nq + t) * N, c0, reinterpret_cast<u64*>(sh[hs]), ar, ld, tid, act);
    return;
  }
  by -= nint;
  const int npair = (tg.n + 1) >> 1;
  const int p = by / npair, pr = by - p * npair;
  const int t0 = tg.t[2 * pr];
  const bool has1 = 2 * pr + 1 < tg.n;
  const int t1 = has1 ? tg.t[2 * pr + 1] : t0;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, hl = lane >> 5, i = lane & 31;
  const int tid = 32 * wave + i;  // the column-pass thread this lane stands for
  const int t = hl ? t1 : t0;
  const ModConst mk = mc[t];
  const F64LazyArith ar{twf + (size_t)t * N, mk.qf, mk.qinvf, (double)mk.ninv};
  double* tile = sh[hl];
  {
    const int ta = ((i >> 2) & 1) ? t1 : t0, j = (i & 3) + 4 * (i >> 3);
    long aop[KW / 2];
#pragma unroll
    for (int m = 0; m < KW / 2; m++) aop[m] = i < 16 ? (long)cdig[((size_t)ta * 8 + j) * KW + 2 * m + hl] : 0;
    const u64* rec = V + (size_t)p * KU * N;
#pragma unroll
    for (int k = 0; k < ITA; k++) {
      const int it = tid + TPB * k, c = it % C, rl = it / C;
      double v[16];
#pragma unroll
      for (int m0 = 0; m0 < NA; m0 += 4) {
        long b[4][KW / 2];
#pragma unroll
        for (int u = 0; u < 4; u++) {
          const size_t idx = (size_t)(rl + ((m0 + u) << GB)) * T1 + c0 + c;
#pragma unroll
          for (int m = 0; m < KW / 2; m++) {
            if (2 * m + 1 < KU) {
              b[u][m] = (long)rec[(size_t)(2 * m + hl) * N + idx];
            } else {  // the last step's upper word is padding: zero in lanes 32..63
              const long w = (long)rec[(size_t)(2 * m) * N + idx];
              b[u][m] = hl ? 0 : w;
            }
          }
        }
#pragma unroll
        for (int u = 0; u < 4; u++) {
          mfma_i32x16 acc = {};
#pragma unroll
          for (int m = 0; m < KW / 2; m++)
            acc = __builtin_amdgcn_mfma_i32_32x32x16_i8(aop[m], b[u][m], acc, 0, 0, 0);
          // sum_j S_j 2^(7 j) = P_hi 2^21 + P_lo, S_j < 2^19.2: the 32-bit
          // pairs S_2m + 2^7 S_(2m+1) < 2^26.3, then P_hi < q (the digits of
          // a constant below q end below bit log2 q) and P_lo < 2^33.3, both
          // exact; one signed product by 2^21 and one centring
          const int s01 = acc[0] + (acc[1] << 7), s34 = acc[3] + (acc[4] << 7), s56 = acc[5] + (acc[6] << 7);
          const double ph = (double)s56 * 0x1p14 + (double)s34;
          const double pl = (double)acc[2] * 0x1p14 + (double)s01;
          v[m0 + u] = f64_centre(f64_mulmod_signed(ph, 0x1p21, ar.q, ar.qinv) + pl, ar.q, ar.qinv);
        }
      }
      fwd_group<GA>(v, 0, 0u, ar);
#pragma unroll
      for (int mm = 0; mm < NA; mm++) tile[lds_rc(rl + (mm << GB), c, C)] = v[mm];
    }
  }
  __syncthreads();
  // second group: r bits [0, GB) -> stages GA..S1-1; y stored packed (the
  // block pass reads it with LoadPacked)
  const bool store = !hl || has1;
  u32* lo = reinterpret_cast<u32*>(y + ((size_t)p * nq + t) * N);
  u8* hi1 = reinterpret_cast<u8*>(lo + N);
  u16* hi2 = reinterpret_cast<u16*>(lo + N);
  const bool hb1 = mk.bits <= 40;
#pragma unroll
  for (int k = 0; k < ITB; k++) {
    const int it = tid + TPB * k, c = it % C, rh = it / C;
    double v[16];
#pragma unroll
    for (int mm = 0; mm < (1 << GB); mm++) v[mm] = tile[lds_rc((rh << GB) + mm, c, C)];
    fwd_group<GB>(v, GA, (u32)rh, ar);
    if (store)
#pragma unroll
      for (int mm = 0; mm < (1 << GB); mm++) {
        const size_t idx = (size_t)((rh << GB) + mm) * T1 + c0 + c;
        const u64 w = ar.store(v[mm]);
        lo[idx] = (u32)w;
        if (hb1) hi1[idx] = (u8)(w >> 32);
        else hi2[idx] = (u16)(w >> 32);
      }
  }
}

template <int LOGN, int GA, int GB, int GC, int GD>
static void moddown_fused(const DeviceTables& T, u64* y, const u64* V, const FbcArgs& A, int nq, int npoly,
                          const LimbMap& map, const u64* x, int x_stride, const u64* pinv, u64* out, hipStream_t s,
                          const u64* cdig, bool pack_out) {
  constexpr int R = 1 << (GA + GB), C = TILE / R;
  {
    ProfScope ps("ntt_fwd_cols_fbc", s, 8.0 * T.N * npoly * ((double)A.ns + 1 + nq),
                 mm_q(T, nq, 0.5 * T.N * (GA + GB) + (double)T.N * (A.ns + 1), npoly));
    if (!cdig) {
      dim3 gc((1 << LOGN) / R / C, nq * npoly);
      hipLaunchKernelGGL((k_ntt_cols2_fbc<LOGN, GA, GB>), gc, dim3(TPB), 0, s, y, V, nq, A, T.psi, T.psi_sh,
                         T.psi_f, T.nmods, T.mc);
    } else {
      // FP64 targets in pairs through the MFMA lift, the Shoup-path targets
      // (above 46 bits) two units a work-group, in one launch
      FbcTgts f, o;
      f.n = o.n = 0;
      for (int t = 0; t < nq; t++) {
        if (T.bits[t] <= F64_LAZY_BITS) f.t[f.n++] = (short)t;
        else o.t[o.n++] = (short)t;
      }
      const int gy = (o.n * npoly + 1) / 2 + ((f.n + 1) / 2) * npoly;
      auto go = [&](auto ns) {
        constexpr int NS = decltype(ns)::value;
        hipLaunchKernelGGL((k_ntt_cols2_fbc_mfma<LOGN, GA, GB, NS>), dim3((1 << LOGN) / R / C, gy), dim3(2 * TPB), 0,
                           s, y, V, nq, npoly, f, o, A, cdig, T.psi, T.psi_sh, T.psi_f, T.nmods, T.mc,
                           g_knobs.xcd_map);
      };
      switch (A.ns) {
        case 1: go(std::integral_constant<int, 1>{}); break;
        case 2: go(std::integral_constant<int, 2>{}); break;
        case 3: go(std::integral_constant<int, 3>{}); break;
        default: go(std::integral_constant<int, 4>{}); break;
      }
    }
  }
  ntt2_fwd_sub<LOGN, GA, GB, GC, GD>(T, y, nq, npoly, map, x, x_stride, pinv, out, s, false, cdig != nullptr,
                                     pack_out);
}
// ModDown of npoly polynomials: xp_coef their P limbs in the coefficient
// domain [npoly][ns][N], x the R_{Q_l P} data ([npoly][x_stride][N]), out
// [npoly][nq][N]; false when the ring size has no register-blocked NTT
static FbcArgs fbc_args(const FbcTable& tab, int src_stride, int src_off) {
  FbcArgs A;
  A.ns = tab.ns;
  A.src_stride = src_stride;
  A.src_off = src_off;
  for (int a = 0; a < tab.ns; a++) {
    A.src[a] = tab.src[a];
    A.hatinv[a] = tab.hatinv[a];
    A.hatinv_sh[a] = tab.hatinv_sh[a];
    A.qrecip[a] = 1.0 / tab.qd[a];
    for (int w = 0; w < 4; w++) A.Hw[a][w] = tab.Hw[a][w];
  }
  for (int w = 0; w < 4; w++) A.Dw[w] = tab.Dw[w];
  A.hat_t = tab.hat_t;
  A.hat_t_sh = tab.hat_t_sh;
  A.D_mod_t = tab.D_mod_t;
  A.hat_f = tab.hat_f;
  return A;
}
// the MFMA lift takes targets of 33 to 46 bits and, beside them, Shoup-path
// targets above 46 bits
bool fbc_digit_path(const DeviceTables& T, const FbcTable& tab, int nq) {
  if (!g_knobs.fbc_mfma || !tab.cdig || tab.kw <= 0 || nq > 64 || tab.ns > 4 || T.logN < 12 || T.logN > 16)
    return false;
  for (int t = 0; t < nq; t++)
    if (T.bits[t] <= 32) return false;
  return true;
}
bool launch_moddown_fused(const DeviceTables& T, const u64* xp_coef, int nq, int npoly, const FbcTable& tab,
                          const u64* x, int x_stride, const u64* pinv, u64* out, u64* y, u64* V, hipStream_t s,
                          int src_stride, int src_off, bool v_ready, bool pack_out) {
  if (T.logN < 12 || T.logN > 16 || tab.ns > 4) return false;
  const FbcArgs A = fbc_args(tab, src_stride > 0 ? src_stride : tab.ns, src_stride > 0 ? src_off : 0);
  const u64* cdig = fbc_digit_path(T, tab, nq) ? tab.cdig : nullptr;
  if (v_ready && !cdig) throw std::runtime_error("digit records given where the ModDown does not take them");
  if (!v_ready) {
    Mm mm;
    for (int a = 0; a < tab.ns; a++) mm.add(T.bits[tab.src[a]], (double)T.N * npoly);
    ProfScope ps("fbc_prep", s, 8.0 * T.N * npoly * (2.0 * tab.ns + 1), mm);
    dim3 gp(cdiv(T.N, TPB), npoly);
    if (!cdig) hipLaunchKernelGGL(k_fbc_prep, gp, dim3(TPB), 0, s, V, xp_coef, A, T.logN, T.mc);
    else if (tab.ns == 1) hipLaunchKernelGGL(k_fbc_prep_digits<1>, gp, dim3(TPB), 0, s, V, xp_coef, A, T.logN, T.mc);
    else if (tab.ns == 2) hipLaunchKernelGGL(k_fbc_prep_digits<2>, gp, dim3(TPB), 0, s, V, xp_coef, A, T.logN, T.mc);
    else if (tab.ns == 3) hipLaunchKernelGGL(k_fbc_prep_digits<3>, gp, dim3(TPB), 0, s, V, xp_coef, A, T.logN, T.mc);
    else hipLaunchKernelGGL(k_fbc_prep_digits<4>, gp, dim3(TPB), 0, s, V, xp_coef, A, T.logN, T.mc);
  }
  LimbMap map;
  map.n = nq;
  for (int k = 0; k < nq; k++) map.idx[k] = (short)k;
  return ntt_dispatch(T.logN, [&](auto sp) {
    using S = decltype(sp);
    moddown_fused<NTT_SPLIT_ARGS>(T, y, V, A, nq, npoly, map, x, x_stride, pinv, out, s, cdig, pack_out);
  });
}


// out[p][t] = (x[p][t] - y[p][t]) * P^{-1} mod q_t   (p < npoly, t < nq)
__global__ void k_moddown_final(u64* out, const u64* x, const u64* y, int nq, const u64* pinv, int x_stride_limbs,
                                int logN, const ModConst* __restrict__ mc) {
  const u64 N = 1ull << logN;
  u32 i = blockIdx.x * TPB + threadIdx.x;
  int t = blockIdx.y, p = blockIdx.z;
  if (i >= N) return;
  u64 q = mc[t].q;
  u64 d = sub_mod(x[((size_t)p * x_stride_limbs + t) * N + i], y[((size_t)p * nq + t) * N + i], q);
  out[((size_t)p * nq + t) * N + i] = mul_const_any(d, pinv[2 * t], pinv[2 * t + 1], mc[t]);
}
void launch_moddown_final(const DeviceTables& T, u64* out, const u64* x, const u64* y, int nq, const u64* pinv,
                          int npoly, int x_stride_limbs, hipStream_t s) {
  ProfScope ps("moddown_final", s, 8.0 * T.N * 3.0 * npoly * nq, mm_q(T, nq, (double)T.N, npoly));
  dim3 grid(cdiv(T.N, TPB), nq, npoly);
  hipLaunchKernelGGL(k_moddown_final, grid, dim3(TPB), 0, s, out, x, y, nq, pinv, x_stride_limbs, T.logN, T.mc);
}

// Hoisted rotation in R_{Q_l P} of MB batch members sharing one key: for each
// limb pos and both key halves,
//   out_b = sum_j pi_g(d_{b,j}) * swk_j  (+ P * pi_g(c0_b) on the Q limbs of the b half)
// Each key word is read once and applied to every member.
// digits [B][beta][nqp][N], c0 [B][nq][N], out [2][B][nqp][N]
#define MS_MAXB 8
// Key inner product of MB members, reduced once per output:
//  * FP64 (q < 2^46): the beta <= 16 signed products a w - k q (each below q
//    in absolute value) sum exactly in a double and one f64_canon reduces
//    the sum;
//  * integer: the 128-bit products are summed (beta terms of < 2^122 fit in
//    128 bits) and the sum is reduced once: hi 2^64 + lo = hi (2^64 mod q) + lo.
// Both equal sum_j d_j key_j mod q exactly.
struct U128 {
  u64 lo, hi;
};
__device__ __forceinline__ void u128_mac(U128& acc, u64 a, u64 b) {
  const u64 lo = a * b, hi = mulhi64(a, b);
  const u64 s = acc.lo + lo;
  acc.hi += hi + (s < lo);
  acc.lo = s;
}
__device__ __forceinline__ u64 u128_reduce(const U128& x, const ModConst& m) {
  const u64 h = reduce64(x.hi, m);
  return add_mod(mul_mod(h, m.r64, m), reduce64(x.lo, m), m.q);
}

// streaming accesses: each key word and each output word is touched once, so
// they are loaded and stored non-temporally and leave L2 to the digits,
// which every rotation of a launch reads again
__device__ __forceinline__ u64 ldnt(const u64* p) { return __builtin_nontemporal_load(p); }
__device__ __forceinline__ void stnt(u64* p, u64 v) { __builtin_nontemporal_store(v, p); }

template <int MB, bool F64>
__device__ __forceinline__ void multsum_body(u64* out, const u64* __restrict__ digits, const u64* __restrict__ key,
                                             const u64* __restrict__ c0, const u64* __restrict__ pmod, int nq,
                                             int nqp, int beta, int nmods, int B, int b0, int m, int pos, u32 i,
                                             u32 src, u64 N, const ModConst& mk,
                                             const u64* __restrict__ mask = nullptr, bool accumulate = false) {
  const size_t dstride = (size_t)beta * nqp * N;
  u64 r0[MB], r1[MB];
  if (F64) {
    const double q = mk.qf, qi = mk.qinvf;
    double s0[MB], s1[MB];
#pragma unroll
    for (int b = 0; b < MB; b++) s0[b] = s1[b] = 0.0;
    // software-pipelined: the loads of digit j + 1 are in flight while j is multiplied
    u64 kbn = ldnt(&key[((size_t)0 * nmods + m) * N + i]), kan = ldnt(&key[((size_t)1 * nmods + m) * N + i]), dn[MB];
#pragma unroll
    for (int b = 0; b < MB; b++) dn[b] = digits[(size_t)(b0 + b) * dstride + (size_t)pos * N + src];
    for (int j = 0; j < beta; j++) {
      // FP64 limbs of a switching key hold doubles (launch_key_f64)
      const double kb = __longlong_as_double((long long)kbn), ka = __longlong_as_double((long long)kan);
      double d[MB];
#pragma unroll
      for (int b = 0; b < MB; b++) d[b] = __longlong_as_double((long long)dn[b]);  // centred double digits
      if (j + 1 < beta) {
        kbn = ldnt(&key[(((size_t)(j + 1) * 2 + 0) * nmods + m) * N + i]);
        kan = ldnt(&key[(((size_t)(j + 1) * 2 + 1) * nmods + m) * N + i]);
#pragma unroll
        for (int b = 0; b < MB; b++)
          dn[b] = digits[(size_t)(b0 + b) * dstride + ((size_t)(j + 1) * nqp + pos) * N + src];
      }
#pragma unroll
      for (int b = 0; b < MB; b++) {
        s0[b] += f64_mulmod_signed(d[b], kb, q, qi);
        s1[b] += f64_mulmod_signed(d[b], ka, q, qi);
      }
    }
#pragma unroll
    for (int b = 0; b < MB; b++) {
      r0[b] = d2u(f64_canon(s0[b], q, qi));
      r1[b] = d2u(f64_canon(s1[b], q, qi));
    }
  } else {
    U128 s0[MB], s1[MB];
#pragma unroll
    for (int b = 0; b < MB; b++) s0[b] = s1[b] = U128{0, 0};
    u64 kbn = ldnt(&key[((size_t)0 * nmods + m) * N + i]), kan = ldnt(&key[((size_t)1 * nmods + m) * N + i]), dn[MB];
#pragma unroll
    for (int b = 0; b < MB; b++) dn[b] = digits[(size_t)(b0 + b) * dstride + (size_t)pos * N + src];
    for (int j = 0; j < beta; j++) {
      const u64 kb = kbn, ka = kan;
      u64 d[MB];
#pragma unroll
      for (int b = 0; b < MB; b++) d[b] = dn[b];
      if (j + 1 < beta) {
        kbn = ldnt(&key[(((size_t)(j + 1) * 2 + 0) * nmods + m) * N + i]);
        kan = ldnt(&key[(((size_t)(j + 1) * 2 + 1) * nmods + m) * N + i]);
#pragma unroll
        for (int b = 0; b < MB; b++)
          dn[b] = digits[(size_t)(b0 + b) * dstride + ((size_t)(j + 1) * nqp + pos) * N + src];
      }
#pragma unroll
      for (int b = 0; b < MB; b++) {
        u128_mac(s0[b], d[b], kb);
        u128_mac(s1[b], d[b], ka);
      }
    }
#pragma unroll
    for (int b = 0; b < MB; b++) {
      r0[b] = u128_reduce(s0[b], mk);
      r1[b] = u128_reduce(s1[b], mk);
    }
  }
  // optional epilogue: out (+)= mask (.) rotation, the mask a plaintext in
  // R_{Q_l P} broadcast over members and both halves
  const u64 mv = mask ? mask[(size_t)pos * N + i] : 0;
#pragma unroll
  for (int b = 0; b < MB; b++) {
    if (c0 && pos < nq) {
      const u64 v = c0[((size_t)(b0 + b) * nq + pos) * N + src];
      r0[b] = add_mod(r0[b], mul_const_any(v, pmod[2 * m], pmod[2 * m + 1], mk), mk.q);
    }
    u64* o0 = &out[((size_t)(b0 + b) * nqp + pos) * N + i];
    u64* o1 = &out[((size_t)(B + b0 + b) * nqp + pos) * N + i];
    if (mask) {
      r0[b] = mul_mod_any(r0[b], mv, mk);
      r1[b] = mul_mod_any(r1[b], mv, mk);
      if (accumulate) {
        r0[b] = add_mod(r0[b], *o0, mk.q);
        r1[b] = add_mod(r1[b], *o1, mk.q);
      }
    }
    stnt(o0, r0[b]);
    stnt(o1, r1[b]);
  }
}

template <int MB>
__global__ void __launch_bounds__(TPB) k_multsum(u64* out, const u64* __restrict__ digits,
                                                 const u64* __restrict__ key, const u64* __restrict__ c0,
                                                 const u64* __restrict__ pmod, int nq, int nqp, int L, int beta,
                                                 int nmods, int B, int b0, u64 g, int logN,
                                                 const ModConst* __restrict__ mc) {
  const u64 N = 1ull << logN;
  u32 i = blockIdx.x * TPB + threadIdx.x;
  int pos = blockIdx.y;
  if (i >= N) return;
  int m = pos < nq ? pos : L + 1 + (pos - nq);
  const ModConst mk = mc[m];
  u32 src = g == 1 ? i : automorph_src(i, g, logN);
  if (mk.bits <= F64_LAZY_BITS)
    multsum_body<MB, true>(out, digits, key, c0, pmod, nq, nqp, beta, nmods, B, b0, m, pos, i, src, N, mk);
  else
    multsum_body<MB, false>(out, digits, key, c0, pmod, nq, nqp, beta, nmods, B, b0, m, pos, i, src, N, mk);
}
// Several hoisted rotations of one decomposition in one launch.  A
// work-group takes a 256-coefficient block S of the digits and one rotation
// r: the automorphism maps the aligned block S onto an aligned block (it
// permutes inside it), so thread t reads digit s = 256 S + t contiguously and
// produces output i = pi_{g_r}^{-1}(s) with the key read at i.  Work-groups of
// one source block for all rotations are spaced eight apart in dispatch
// order, so they land on the same XCD back to back and the digits come from
// its L2 after the first rotation: HBM reads them once per launch.
struct MultiRot {
  u64* out[MR_MAX];
  const u64* key[MR_MAX];
  const u64* mask[MR_MAX];  // null: plain outputs
  u64 ginv[MR_MAX];
  int accumulate;           // with masks: add onto the outputs
  // a second base under the same keys (pair launches): its digits, c0 and
  // masks; each output is mask (first) + mask2 (second)
  const u64* digits2;
  const u64* c02;
  const u64* mask2[MR_MAX];
};
// Limbs of R_{Q_l P} in launch order: the integer limbs (moduli of 47 bits
// or more, four members at a time to bound their registers) are spread
// among the FP64 ones so that their VALU-heavy blocks overlap the others.
struct PosList {
  short pos[HE_MAXMOD];
};
// RPW rotations r0 .. r0 + nr - 1 (nr <= RPW) of one decomposition at one
// FP64 limb for one thread: the thread's digits (and c0) are read once and
// serve every rotation of the group, each with its own key, output index
// and epilogue.  The sums are those of multsum_body, term for term.
template <int MB, int RPW>
__device__ __forceinline__ void multsum_rot_group(const MultiRot& R, int r0, int nr, const u64* __restrict__ digits,
                                                  const u64* __restrict__ c0, const u64* __restrict__ pmod, int nq,
                                                  int nqp, int beta, int nmods, int B, int b0, int m, int pos,
                                                  u32 src, int logN, u64 N, const ModConst& mk) {
  const size_t dstride = (size_t)beta * nqp * N;
  const double q = mk.qf, qi = mk.qinvf;
  u32 idx[RPW];
  const u64* key[RPW];
#pragma unroll
  for (int g = 0; g < RPW; g++) {
    const int r = r0 + (g < nr ? g : 0);  // past nr: a duplicate of the first, never stored
    idx[g] = automorph_src(src, R.ginv[r], logN);
    key[g] = R.key[r];
  }
  double s0[RPW][MB], s1[RPW][MB];
#pragma unroll
  for (int g = 0; g < RPW; g++)
#pragma unroll
    for (int b = 0; b < MB; b++) s0[g][b] = s1[g][b] = 0.0;
  // software-pipelined as multsum_body: digit j + 1 and the keys at j + 1 in
  // flight while j is multiplied
  u64 kbn[RPW], kan[RPW], dn[MB];
#pragma unroll
  for (int g = 0; g < RPW; g++) {
    kbn[g] = ldnt(&key[g][((size_t)0 * nmods + m) * N + idx[g]]);
    kan[g] = ldnt(&key[g][((size_t)1 * nmods + m) * N + idx[g]]);
  }
#pragma unroll
  for (int b = 0; b < MB; b++) dn[b] = digits[(size_t)(b0 + b) * dstride + (size_t)pos * N + src];
  for (int j = 0; j < beta; j++) {
    double kb[RPW], ka[RPW], d[MB];
#pragma unroll
    for (int g = 0; g < RPW; g++) {
      kb[g] = __longlong_as_double((long long)kbn[g]);  // key limbs stored as doubles
      ka[g] = __longlong_as_double((long long)kan[g]);
    }
#pragma unroll
    for (int b = 0; b < MB; b++) d[b] = __longlong_as_double((long long)dn[b]);  // centred double digits
    if (j + 1 < beta) {
#pragma unroll
      for (int g = 0; g < RPW; g++) {
        kbn[g] = ldnt(&key[g][(((size_t)(j + 1) * 2 + 0) * nmods + m) * N + idx[g]]);
        kan[g] = ldnt(&key[g][(((size_t)(j + 1) * 2 + 1) * nmods + m) * N + idx[g]]);
      }
#pragma unroll
      for (int b = 0; b < MB; b++) dn[b] = digits[(size_t)(b0 + b) * dstride + ((size_t)(j + 1) * nqp + pos) * N + src];
    }
#pragma unroll
    for (int g = 0; g < RPW; g++)
#pragma unroll
      for (int b = 0; b < MB; b++) {
        s0[g][b] += f64_mulmod_signed(d[b], kb[g], q, qi);
        s1[g][b] += f64_mulmod_signed(d[b], ka[g], q, qi);
      }
  }
  // c0 P on the Q limbs, once for the group.  The epilogue stays in the
  // lazy FP64 domain: a sum of beta terms below q in absolute value, plus
  // c0 P in [0, q), is within 16 q for beta <= 15 (centred first otherwise),
  // so the mask product applies to it directly; with the old output added the
  // value is within 2 q, and one reduction gives the residue in [0, q).
  double cpd[MB];
#pragma unroll
  for (int b = 0; b < MB; b++)
    cpd[b] = (c0 && pos < nq)
                 ? u2d(mul_const_any(c0[((size_t)(b0 + b) * nq + pos) * N + src], pmod[2 * m], pmod[2 * m + 1], mk))
                 : 0.0;
#pragma unroll
  for (int g = 0; g < RPW; g++) {
    if (g >= nr) break;
    const int r = r0 + g;
    const u64* mask = R.mask[r];
    const u32 i = idx[g];
    const double mv = mask ? u2d(mask[(size_t)pos * N + i]) : 0.0;
#pragma unroll
    for (int b = 0; b < MB; b++) {
      double a0 = s0[g][b] + cpd[b], a1 = s1[g][b];
      u64* o0 = &R.out[r][((size_t)(b0 + b) * nqp + pos) * N + i];
      u64* o1 = &R.out[r][((size_t)(B + b0 + b) * nqp + pos) * N + i];
      if (mask) {
        if (beta > 15) {
          a0 = f64_centre(a0, q, qi);
          a1 = f64_centre(a1, q, qi);
        }
        a0 = f64_mulmod_signed(a0, mv, q, qi);
        a1 = f64_mulmod_signed(a1, mv, q, qi);
        if (R.accumulate) {
          a0 += u2d(*o0);
          a1 += u2d(*o1);
        }
      }
      stnt(o0, d2u(f64_canon(a0, q, qi)));
      stnt(o1, d2u(f64_canon(a1, q, qi)));
    }
  }
}
// The same for two bases under the same keys (pair launches): the digits of
// base 1 (digits, c0, masks) and base 2 (R.digits2, R.c02, R.mask2) as 2 MB
// digit lanes, so that each key word is loaded once for both; the output is
//   mask (sum_1 + c0_1 P) + mask2 (sum_2 + c0_2 P),
// each masked term below q in absolute value, reduced once: the residues of
// the first base's launch followed by the second's accumulating launch.
template <int MB, int RPW>
__device__ __forceinline__ void multsum_rot_group_pair(const MultiRot& R, int r0, int nr,
                                                       const u64* __restrict__ digits, const u64* __restrict__ c0,
                                                       const u64* __restrict__ pmod, int nq, int nqp, int beta,
                                                       int nmods, int B, int b0, int m, int pos, u32 src, int logN,
                                                       u64 N, const ModConst& mk) {
  constexpr int NB = 2 * MB;
  const size_t dstride = (size_t)beta * nqp * N;
  const double q = mk.qf, qi = mk.qinvf;
  u32 idx[RPW];
  const u64* key[RPW];
#pragma unroll
  for (int g = 0; g < RPW; g++) {
    const int r = r0 + (g < nr ? g : 0);
    idx[g] = automorph_src(src, R.ginv[r], logN);
    key[g] = R.key[r];
  }
  const u64* dg[2] = {digits, R.digits2};
  double s0[RPW][NB], s1[RPW][NB];
#pragma unroll
  for (int g = 0; g < RPW; g++)
#pragma unroll
    for (int b = 0; b < NB; b++) s0[g][b] = s1[g][b] = 0.0;
  u64 kbn[RPW], kan[RPW], dn[NB];
#pragma unroll
  for (int g = 0; g < RPW; g++) {
    kbn[g] = ldnt(&key[g][((size_t)0 * nmods + m) * N + idx[g]]);
    kan[g] = ldnt(&key[g][((size_t)1 * nmods + m) * N + idx[g]]);
  }
#pragma unroll
  for (int b = 0; b < NB; b++) dn[b] = dg[b / MB][(size_t)(b0 + b % MB) * dstride + (size_t)pos * N + src];
  for (int j = 0; j < beta; j++) {
    double kb[RPW], ka[RPW], d[NB];
#pragma unroll
    for (int g = 0; g < RPW; g++) {
      kb[g] = __longlong_as_double((long long)kbn[g]);  // key limbs stored as doubles
      ka[g] = __longlong_as_double((long long)kan[g]);
    }
#pragma unroll
    for (int b = 0; b < NB; b++) d[b] = __longlong_as_double((long long)dn[b]);  // centred double digits
    if (j + 1 < beta) {
#pragma unroll
      for (int g = 0; g < RPW; g++) {
        kbn[g] = ldnt(&key[g][(((size_t)(j + 1) * 2 + 0) * nmods + m) * N + idx[g]]);
        kan[g] = ldnt(&key[g][(((size_t)(j + 1) * 2 + 1) * nmods + m) * N + idx[g]]);
      }
#pragma unroll
      for (int b = 0; b < NB; b++)
        dn[b] = dg[b / MB][(size_t)(b0 + b % MB) * dstride + ((size_t)(j + 1) * nqp + pos) * N + src];
    }
#pragma unroll
    for (int g = 0; g < RPW; g++)
#pragma unroll
      for (int b = 0; b < NB; b++) {
        s0[g][b] += f64_mulmod_signed(d[b], kb[g], q, qi);
        s1[g][b] += f64_mulmod_signed(d[b], ka[g], q, qi);
      }
  }
  const u64* cs[2] = {c0, R.c02};
  double cpd[NB];
#pragma unroll
  for (int b = 0; b < NB; b++)
    cpd[b] = pos < nq ? u2d(mul_const_any(cs[b / MB][((size_t)(b0 + b % MB) * nq + pos) * N + src], pmod[2 * m],
                                          pmod[2 * m + 1], mk))
                      : 0.0;
#pragma unroll
  for (int g = 0; g < RPW; g++) {
    if (g >= nr) break;
    const int r = r0 + g;
    const u32 i = idx[g];
    const double mv1 = u2d(R.mask[r][(size_t)pos * N + i]), mv2 = u2d(R.mask2[r][(size_t)pos * N + i]);
#pragma unroll
    for (int b = 0; b < MB; b++) {
      double a0 = s0[g][b] + cpd[b], a1 = s1[g][b], e0 = s0[g][MB + b] + cpd[MB + b], e1 = s1[g][MB + b];
      if (beta > 15) {
        a0 = f64_centre(a0, q, qi);
        a1 = f64_centre(a1, q, qi);
        e0 = f64_centre(e0, q, qi);
        e1 = f64_centre(e1, q, qi);
      }
      a0 = f64_mulmod_signed(a0, mv1, q, qi) + f64_mulmod_signed(e0, mv2, q, qi);
      a1 = f64_mulmod_signed(a1, mv1, q, qi) + f64_mulmod_signed(e1, mv2, q, qi);
      stnt(&R.out[r][((size_t)(b0 + b) * nqp + pos) * N + i], d2u(f64_canon(a0, q, qi)));
      stnt(&R.out[r][((size_t)(B + b0 + b) * nqp + pos) * N + i], d2u(f64_canon(a1, q, qi)));
    }
  }
}
// Key inner products on the 60-bit limbs (q0 and the special primes), where
// the lazy FP64 product does not apply.  Each product d k is taken apart into
// 20-bit pieces, d = d0 + d1 2^20 + d2 2^40 and k likewise, and the nine
// piece products (below 2^42 for residues below 2^61) are summed with FMAs
// into five sums by weight 2^(20 w): S_w holds at most 3 beta of them, below
// 2^50 for beta <= 64, so every FMA is exact.  The sum over the digits is
// X = sum_w S_w 2^(20 w) < beta 2^122 <= 2^128, the same integer the 128-bit
// multiply-accumulate forms, and it is reduced once, so the residues are
// those of the integer products.  Nine full-rate FP64 FMAs take the place of
// four quarter-rate 32-bit multiplies and the carries of a 128-bit sum.
// Each digit is taken apart once for both key halves; members go four at a
// time (2 x 4 x 5 sums).
constexpr u64 PIECE20 = (1ull << 20) - 1;
__device__ __forceinline__ void split20(u64 x, double& x0, double& x1, double& x2) {
  x0 = u2d(x & PIECE20);
  x1 = u2d((x >> 20) & PIECE20);
  x2 = u2d(x >> 40);
}
// x = hi 2^64 + lo (hi < 2^62) mod q for 2^46 < q < 2^61: the high word's
// halves are folded with 2^96 and 2^64 mod q into Y < 2^95, Y's quotient by q
// (below 2^49) is estimated in FP64, off by at most one since Y's relative
// rounding is 2^-51, and the remainder, in (-q, 2q), is computed in 64-bit
// words and corrected once.
__device__ __forceinline__ u64 reduce128_est(u64 lo, u64 hi, const ModConst& m) {
  u64 y0 = lo, y1 = 0;
  auto mac = [&](u64 a, u64 r) {  // (y1, y0) += a r, a < 2^32
    const u64 l = a * (r & 0xffffffffull), h = a * (r >> 32);
    const u64 hl = h << 32;
    u64 s = y0 + l;
    y1 += (s < l ? 1 : 0) + (h >> 32);
    y0 = s + hl;
    y1 += y0 < hl ? 1 : 0;
  };
  mac(hi >> 32, m.r96);
  mac(hi & 0xffffffffull, m.r64);
  const double yd = __fma_rn((double)y1, 0x1p64, (double)y0);
  const u64 k = (u64)__builtin_floor(yd * m.qinvf);
  long long r = (long long)(y0 - k * m.q);
  if (r < 0) r += (long long)m.q;
  else if ((u64)r >= m.q) r -= (long long)m.q;
  return (u64)r;
}
__device__ __forceinline__ u64 fold_pieces(const double* S, const ModConst& mk) {
  u64 lo = d2u(S[0]), hi = 0;
#pragma unroll
  for (int w = 1; w < 5; w++) {
    const u64 v = d2u(S[w]);
    const int sh = 20 * w;
    const u64 l = sh < 64 ? v << sh : 0, h = sh < 64 ? v >> (64 - sh) : v << (sh - 64);
    lo += l;
    hi += h + (lo < l ? 1 : 0);
  }
  return reduce128_est(lo, hi, mk);
}
template <int MB>
__device__ __forceinline__ void multsum_int_pass(const MultiRot& R, int r, u32 i, const u64* __restrict__ dig,
                                                 size_t dstride, size_t jstride, const u64* __restrict__ c0,
                                                 const u64* __restrict__ pmod, int nq, int nqp, int beta, int nmods,
                                                 int B, int b0, int m, int pos, u32 src, u64 N, const ModConst& mk) {
  const u64* key = R.key[r];
  double S0[MB][5], S1[MB][5];
#pragma unroll
  for (int b = 0; b < MB; b++)
#pragma unroll
    for (int w = 0; w < 5; w++) S0[b][w] = S1[b][w] = 0.0;
  // software-pipelined: the key words and digits of j + 1 are in flight
  // while j is multiplied.  Plain loads: the keys are read again by the
  // next pass over the members, from L2.
  u64 kbn = key[(size_t)m * N + i], kan = key[((size_t)nmods + m) * N + i], dn[MB];
#pragma unroll
  for (int b = 0; b < MB; b++) dn[b] = dig[(size_t)b * dstride];
  for (int j = 0; j < beta; j++) {
    double kb0, kb1, kb2, ka0, ka1, ka2;
    split20(kbn, kb0, kb1, kb2);
    split20(kan, ka0, ka1, ka2);
    u64 dw[MB];
#pragma unroll
    for (int b = 0; b < MB; b++) dw[b] = dn[b];
    if (j + 1 < beta) {
      kbn = key[(((size_t)(j + 1) * 2 + 0) * nmods + m) * N + i];
      kan = key[(((size_t)(j + 1) * 2 + 1) * nmods + m) * N + i];
#pragma unroll
      for (int b = 0; b < MB; b++) dn[b] = dig[(size_t)b * dstride + (size_t)(j + 1) * jstride];
    }
#pragma unroll
    for (int b = 0; b < MB; b++) {
      double d0, d1, d2;
      split20(dw[b], d0, d1, d2);
      S0[b][0] = fma(d0, kb0, S0[b][0]);
      S0[b][1] = fma(d0, kb1, S0[b][1]);
      S0[b][1] = fma(d1, kb0, S0[b][1]);
      S0[b][2] = fma(d0, kb2, S0[b][2]);
      S0[b][2] = fma(d1, kb1, S0[b][2]);
      S0[b][2] = fma(d2, kb0, S0[b][2]);
      S0[b][3] = fma(d1, kb2, S0[b][3]);
      S0[b][3] = fma(d2, kb1, S0[b][3]);
      S0[b][4] = fma(d2, kb2, S0[b][4]);
      S1[b][0] = fma(d0, ka0, S1[b][0]);
      S1[b][1] = fma(d0, ka1, S1[b][1]);
      S1[b][1] = fma(d1, ka0, S1[b][1]);
      S1[b][2] = fma(d0, ka2, S1[b][2]);
      S1[b][2] = fma(d1, ka1, S1[b][2]);
      S1[b][2] = fma(d2, ka0, S1[b][2]);
      S1[b][3] = fma(d1, ka2, S1[b][3]);
      S1[b][3] = fma(d2, ka1, S1[b][3]);
      S1[b][4] = fma(d2, ka2, S1[b][4]);
    }
  }
  const u64* mask = R.mask[r];
  const u64 mv = mask ? mask[(size_t)pos * N + i] : 0;
#pragma unroll
  for (int b = 0; b < MB; b++) {
    u64 v0 = fold_pieces(S0[b], mk), v1 = fold_pieces(S1[b], mk);
    if (c0 && pos < nq)
      v0 = add_mod(v0, mul_const_any(c0[((size_t)(b0 + b) * nq + pos) * N + src], pmod[2 * m], pmod[2 * m + 1], mk),
                   mk.q);
    u64* o0 = &R.out[r][((size_t)(b0 + b) * nqp + pos) * N + i];
    u64* o1 = &R.out[r][((size_t)(B + b0 + b) * nqp + pos) * N + i];
    if (mask) {
      v0 = mul_mod_any(v0, mv, mk);
      v1 = mul_mod_any(v1, mv, mk);
      if (R.accumulate) {
        v0 = add_mod(v0, *o0, mk.q);
        v1 = add_mod(v1, *o1, mk.q);
      }
    }
    stnt(o0, v0);
    stnt(o1, v1);
  }
}
// MP: members per pass over the digits (4, or all 8 in one pass where the
// launch gives the sums the registers)
template <int MB, int MP = 4>
__device__ __forceinline__ void multsum_rot_group_int(const MultiRot& R, int r0, int nr, const u64* __restrict__ digits,
                                                      const u64* __restrict__ c0, const u64* __restrict__ pmod,
                                                      int nq, int nqp, int beta, int nmods, int B, int b0, int m,
                                                      int pos, u32 src, int logN, u64 N, const ModConst& mk) {
  const size_t dstride = (size_t)beta * nqp * N, jstride = (size_t)nqp * N;
  const u64* dig = digits + (size_t)b0 * dstride + (size_t)pos * N + src;
  constexpr int M1 = MB > MP ? MP : MB;
  for (int r = r0; r < r0 + nr; r++) {
    const u32 i = automorph_src(src, R.ginv[r], logN);
    multsum_int_pass<M1>(R, r, i, dig, dstride, jstride, c0, pmod, nq, nqp, beta, nmods, B, b0, m, pos, src, N, mk);
    if (MB > M1)
      multsum_int_pass<(MB > M1 ? MB - M1 : 1)>(R, r, i, dig + M1 * dstride, dstride, jstride, c0, pmod, nq, nqp,
                                                beta, nmods, B, b0 + M1, m, pos, src, N, mk);
  }
}
// RPW: rotations per work-group (their FP64 limbs share the digit loads)
template <int MB, bool F64, int RPW, bool PAIR = false>
__global__ void __launch_bounds__(TPB) k_multsum_rot(MultiRot R, PosList P, int nrot, const u64* __restrict__ digits,
                                                     const u64* __restrict__ c0, const u64* __restrict__ pmod,
                                                     int nq, int nqp, int L, int beta, int nmods, int B, int b0,
                                                     int logN, const ModConst* __restrict__ mc) {
  const u64 N = 1ull << logN;
  const u32 ngroups = (u32)((nrot + RPW - 1) / RPW);
  const u32 x = blockIdx.x, rest = x >> 3;
  const int r0 = (int)(rest % ngroups) * RPW;
  const int nr = nrot - r0 < RPW ? nrot - r0 : RPW;
  const u32 S = (rest / ngroups) * 8 + (x & 7);
  if ((u64)S * TPB >= N) return;
  const u32 src = S * TPB + threadIdx.x;
  const int pos = P.pos[blockIdx.y];
  const int m = pos < nq ? pos : L + 1 + (pos - nq);
  const ModConst mk = mc[m];
  if (F64 || mk.bits <= F64_LAZY_BITS) {
    if (PAIR)
      multsum_rot_group_pair<MB, RPW>(R, r0, nr, digits, c0, pmod, nq, nqp, beta, nmods, B, b0, m, pos, src, logN, N,
                                      mk);
    else
      multsum_rot_group<MB, RPW>(R, r0, nr, digits, c0, pmod, nq, nqp, beta, nmods, B, b0, m, pos, src, logN, N, mk);
    return;
  }
  multsum_rot_group_int<MB>(R, r0, nr, digits, c0, pmod, nq, nqp, beta, nmods, B, b0, m, pos, src, logN, N, mk);
}

// The 60-bit limbs of a multi-rotation launch on their own (knob
// "mr_int_split"): a kernel without the FP64 group's sums in its registers,
// one rotation per work-group.  Dispatch order: the rotations in chunks of
// rc (knob "mr_int_chunk"); inside a chunk, source blocks in octets, and the
// chunk's rotations of one octet back to back.  Block S goes to XCD S mod 8
// for every rotation, so its digits are read from HBM about once per chunk.
template <int MB, int MP>
__global__ void __launch_bounds__(TPB) k_multsum_rot_int(MultiRot R, PosList P, int nrot, int rc,
                                                         const u64* __restrict__ digits,
                                                         const u64* __restrict__ c0, const u64* __restrict__ pmod,
                                                         int nq, int nqp, int L, int beta, int nmods, int B, int b0,
                                                         int logN, const ModConst* __restrict__ mc) {
  const u64 N = 1ull << logN;
  const u32 x = blockIdx.x, rest = x >> 3;
  const u32 octets = (u32)((N + 8 * TPB - 1) / (8 * TPB));  // source-block octets
  const u32 per_chunk = octets * (u32)rc;
  const u32 chunk = rest / per_chunk, within = rest - chunk * per_chunk;
  const u32 rcc = (u32)(nrot - (int)chunk * rc) < (u32)rc ? (u32)(nrot - (int)chunk * rc) : (u32)rc;
  const int r = (int)(chunk * (u32)rc + within % rcc);
  const u32 S = (within / rcc) * 8 + (x & 7);
  if ((u64)S * TPB >= N) return;
  const u32 src = S * TPB + threadIdx.x;
  const int pos = P.pos[blockIdx.y];
  const int m = pos < nq ? pos : L + 1 + (pos - nq);
  const ModConst mk = mc[m];
  multsum_rot_group_int<MB, MP>(R, r, 1, digits, c0, pmod, nq, nqp, beta, nmods, B, b0, m, pos, src, logN, N, mk);
}

static u64 inv_mod_2n(u64 g, u64 twoN) {
  // g odd: Newton iteration for the inverse modulo a power of two
  u64 x = g;  // correct to 3 bits
  for (int k = 0; k < 6; k++) x *= 2 - g * x;
  return x & (twoN - 1);
}

// Limb order of an R_{Q_l P} element for the key inner products: the integer
// limbs spread among the FP64 ones (see PosList)
static PosList pos_order(const DeviceTables& T, int nq, int nqp, int L) {
  PosList pf, pi, P;
  int nf = 0, ni = 0;
  for (int pos = 0; pos < nqp; pos++) {
    const int m = pos < nq ? pos : L + 1 + (pos - nq);
    if (T.bits[m] <= F64_LAZY_BITS) pf.pos[nf++] = (short)pos;
    else pi.pos[ni++] = (short)pos;
  }
  int f = 0, k = 0;
  for (int t = 0; t < ni; t++) {
    const int upto = (int)(((long)nf * (t + 1)) / (ni + 1));
    while (f < upto) P.pos[k++] = pf.pos[f++];
    P.pos[k++] = pi.pos[t];
  }
  while (f < nf) P.pos[k++] = pf.pos[f++];
  return P;
}

// ---------------------------------------------------------------------------
// Merged key inner products: one launch over a list of work items of any
// level, members and rotations (of different products), read from a device
// table.  Each item runs exactly the arithmetic of k_multsum_rot.
// ---------------------------------------------------------------------------
struct KsItem {
  MultiRot R;
  PosList P;
  const u64* digits;
  const u64* c0;
  const u64* pmod;
  int nrot, nq, nqp, beta, B, b0;
};
constexpr int KS_RPW = 4;  // rotations per work-group in the merged launch
thread_local KsSink* tls_ks_sink = nullptr;
KsSink* ks_sink_exchange(KsSink* s) {
  KsSink* old = tls_ks_sink;
  tls_ks_sink = s;
  return old;
}

template <int MB>
__global__ void __launch_bounds__(TPB) k_multsum_list(const KsItem* __restrict__ items, const u32* __restrict__ start,
                                                      int nitems, int L, int nmods, int logN,
                                                      const ModConst* __restrict__ mc) {
  const u32 x = blockIdx.x;
  int lo = 0, hi = nitems;  // start[lo] <= x < start[lo + 1]
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (start[mid] <= x) lo = mid;
    else hi = mid;
  }
  const KsItem& it = items[lo];
  if ((int)blockIdx.y >= it.nqp) return;
  const u64 N = 1ull << logN;
  const u32 xl = x - start[lo];
  const u32 ngroups = (u32)((it.nrot + KS_RPW - 1) / KS_RPW);
  const u32 rest = xl >> 3;
  const int r0 = (int)(rest % ngroups) * KS_RPW;
  const int nr = it.nrot - r0 < KS_RPW ? it.nrot - r0 : KS_RPW;
  const u32 S = (rest / ngroups) * 8 + (xl & 7);
  if ((u64)S * TPB >= N) return;
  const u32 src = S * TPB + threadIdx.x;
  const int pos = it.P.pos[blockIdx.y];
  const int m = pos < it.nq ? pos : L + 1 + (pos - it.nq);
  const ModConst mk = mc[m];
  if (mk.bits <= F64_LAZY_BITS) {
    multsum_rot_group<MB, KS_RPW>(it.R, r0, nr, it.digits, it.c0, it.pmod, it.nq, it.nqp, it.beta, nmods, it.B,
                                  it.b0, m, pos, src, logN, N, mk);
    return;
  }
  multsum_rot_group_int<MB>(it.R, r0, nr, it.digits, it.c0, it.pmod, it.nq, it.nqp, it.beta, nmods, it.B, it.b0, m,
                            pos, src, logN, N, mk);
}

// the work's items: rotations in chunks of MR_MAX, members in chunks of
// MS_MAXB (an item's member count decides the launch it goes to)
static void ks_items(const DeviceTables& T, const KsWork& w, int L, int alpha, std::vector<std::pair<int, KsItem>>& out) {
  const int nq = w.level + 1, nqp = nq + alpha, nrot = (int)w.gs.size();
  const u64 twoN = 2 * T.N;
  const PosList P = pos_order(T, nq, nqp, L);
  for (int r0 = 0; r0 < nrot; r0 += MR_MAX) {
    const int nr = std::min(nrot - r0, MR_MAX);
    for (int b0 = 0; b0 < w.B; b0 += MS_MAXB) {
      KsItem it;
      std::memset(&it, 0, sizeof it);
      it.R.accumulate = !w.masks.empty() && w.accumulate ? 1 : 0;
      for (int r = 0; r < nr; r++) {
        it.R.out[r] = w.outs[r0 + r];
        it.R.key[r] = w.keys[r0 + r];
        it.R.mask[r] = w.masks.empty() ? nullptr : w.masks[r0 + r];
        it.R.ginv[r] = inv_mod_2n(w.gs[r0 + r], twoN);
      }
      it.P = P;
      it.digits = w.digits;
      it.c0 = w.c0;
      it.pmod = w.pmod;
      it.nrot = nr;
      it.nq = nq;
      it.nqp = nqp;
      it.beta = w.beta;
      it.B = w.B;
      it.b0 = b0;
      out.push_back({std::min(MS_MAXB, w.B - b0), it});
    }
  }
}

// bytes of the table launch_multsum_list lays out: per distinct member count
// a 256-aligned run of items, then a 256-aligned prefix array of its
// work-group counts (one more entry than items)
static size_t ks_table_bytes(std::vector<std::pair<int, KsItem>>& items) {
  std::stable_sort(items.begin(), items.end(), [](const auto& a, const auto& b) { return a.first < b.first; });
  size_t bytes = 0;
  for (size_t i = 0; i < items.size();) {
    size_t j = i;
    while (j < items.size() && items[j].first == items[i].first) j++;
    bytes = ((bytes + 255) & ~(size_t)255) + (j - i) * sizeof(KsItem);
    bytes = ((bytes + 255) & ~(size_t)255) + (j - i + 1) * sizeof(u32);
    i = j;
  }
  return bytes;
}
size_t multsum_list_table_bytes(const DeviceTables& T, const std::vector<KsWork>& works, int L, int alpha) {
  std::vector<std::pair<int, KsItem>> items;
  for (const KsWork& w : works) ks_items(T, w, L, alpha, items);
  return ks_table_bytes(items);
}

void launch_multsum_list(const DeviceTables& T, const std::vector<KsWork>& works, void* table, size_t table_bytes,
                         int L, int alpha, hipStream_t s) {
  std::vector<std::pair<int, KsItem>> items;
  for (const KsWork& w : works) ks_items(T, w, L, alpha, items);
  if (items.empty()) return;
  // one launch per member count: items sorted by it, each group's table
  // (items, then the prefix of their work-group counts) laid out in turn
  const size_t need = ks_table_bytes(items);
  if (need > table_bytes) throw std::runtime_error("merged key-switch table larger than its buffer");
  std::vector<char> host;
  host.reserve(need);
  struct Launch {
    int mb, n, nqp_max;
    size_t items_off, start_off;
    u32 tiles;
    double bytes, unit;
    Mm mm;
  };
  std::vector<Launch> launches;
  const u32 nblk = (u32)cdiv(T.N, TPB), per_rot_group = (u32)cdiv(nblk, 8) * 8;
  for (size_t i = 0; i < items.size();) {
    size_t j = i;
    while (j < items.size() && items[j].first == items[i].first) j++;
    Launch L_;
    L_.mb = items[i].first;
    L_.n = (int)(j - i);
    L_.nqp_max = 0;
    L_.bytes = L_.unit = 0;
    L_.items_off = (host.size() + 255) & ~(size_t)255;
    host.resize(L_.items_off + (size_t)L_.n * sizeof(KsItem));
    std::vector<u32> start;
    u32 t = 0;
    for (size_t k = i; k < j; k++) {
      const KsItem& it = items[k].second;
      std::memcpy(host.data() + L_.items_off + (k - i) * sizeof(KsItem), &it, sizeof(KsItem));
      start.push_back(t);
      t += per_rot_group * (u32)((it.nrot + KS_RPW - 1) / KS_RPW);
      L_.nqp_max = std::max(L_.nqp_max, it.nqp);
      const bool masked = it.R.mask[0] != nullptr;
      const double mb = L_.mb, nr = it.nrot;
      L_.bytes += 8.0 * T.N * it.nqp *
                  (nr * 2.0 * it.beta + mb * it.beta + (masked ? nr : 0.0) + mb * nr * 2.0 * (1 + it.R.accumulate)) +
                  (it.c0 ? 8.0 * T.N * mb * it.nq : 0.0);
      L_.unit += 8.0 * T.N * (nr * 2.0 * it.beta * it.nqp + nr * mb * 4.0 * it.nq);
      L_.mm = L_.mm + mm_qp(T, it.nq, it.nqp, L, (double)T.N * (2.0 * it.beta + (it.c0 ? 1 : 0) + (masked ? 2 : 0)),
                            (double)T.N * (2.0 * it.beta + (masked ? 2 : 0)), mb * nr);
    }
    start.push_back(t);
    L_.tiles = t;
    L_.start_off = (host.size() + 255) & ~(size_t)255;
    host.resize(L_.start_off + start.size() * sizeof(u32));
    std::memcpy(host.data() + L_.start_off, start.data(), start.size() * sizeof(u32));
    launches.push_back(L_);
    i = j;
  }
  if (host.size() != need) throw std::runtime_error("merged key-switch table layout mismatch");
  // pageable source: the copy has read it when the call returns
  if (hipMemcpyAsync(table, host.data(), host.size(), hipMemcpyHostToDevice, s) != hipSuccess)
    throw std::runtime_error("merged key-switch table upload failed");
  for (const Launch& l : launches) {
    const KsItem* it = (const KsItem*)((char*)table + l.items_off);
    const u32* st = (const u32*)((char*)table + l.start_off);
    ProfScope ps("multsum_rot", s, l.bytes, l.mm, l.unit);
    const dim3 grid(l.tiles, l.nqp_max);
#define ML_CASE(K)                                                                                            \
  case K:                                                                                                     \
    hipLaunchKernelGGL(k_multsum_list<K>, grid, dim3(TPB), 0, s, it, st, l.n, L, T.nmods, T.logN, T.mc); \
    break;
    switch (l.mb) { ML_CASE(1) ML_CASE(2) ML_CASE(3) ML_CASE(4) ML_CASE(5) ML_CASE(6) ML_CASE(7) ML_CASE(8) }
#undef ML_CASE
  }
}

// HBM bytes (each rotation's key once, the members' digits and c0 once,
// outputs once, the masks, the outputs read back when accumulating),
// modular products (2 beta key products per member, rotation and value, P c0
// on the Q limbs, the mask on both halves) and key-switch unit bytes of one
// multi-rotation launch over the positions pl[0 .. n)
static void fork_check(hipError_t e, const char* what) {
  if (e != hipSuccess) throw std::runtime_error(std::string("forked stream: ") + what + ": " + hipGetErrorString(e));
}
struct MrCost {
  double bytes = 0, unit = 0;
  Mm mm;
};
static MrCost mr_cost(const DeviceTables& T, const PosList& pl, int n, int nq, int L, int nr, int mb, int beta,
                      bool c0, bool masks, bool acc) {
  MrCost c;
  double w = 0, u = 0;
  for (int x = 0; x < n; x++) {
    const int pos = pl.pos[x];
    const int m = pos < nq ? pos : L + 1 + (pos - nq);
    const bool q = pos < nq;
    w += nr * 2.0 * beta + mb * (beta + (c0 && q ? 1.0 : 0.0) + nr * 2.0) + (masks ? nr : 0.0) +
         (acc ? mb * nr * 2.0 : 0.0);
    c.mm.add(T.bits[m], (double)T.N * (2.0 * beta + (c0 && q ? 1 : 0) + (masks ? 2 : 0)) * mb * nr);
    u += nr * 2.0 * beta + (q ? nr * mb * 4.0 : 0.0);
  }
  c.bytes = 8.0 * T.N * w;
  c.unit = 8.0 * T.N * u;
  return c;
}
void launch_multsum_rot(const DeviceTables& T, u64* const* outs, const u64* const* keys, const u64* gs, int nrot,
                        const u64* digits, const u64* c0, const u64* pmod, int level, int L, int alpha, int beta,
                        int batch, hipStream_t s, const u64* const* masks, bool accumulate,
                        const ForkStream* fs) {
  if (tls_ks_sink) {
    KsWork w;
    w.outs.assign(outs, outs + nrot);
    w.keys.assign(keys, keys + nrot);
    w.gs.assign(gs, gs + nrot);
    if (masks) w.masks.assign(masks, masks + nrot);
    w.accumulate = accumulate;
    w.digits = digits;
    w.c0 = c0;
    w.pmod = pmod;
    w.level = level;
    w.beta = beta;
    w.B = batch;
    (*tls_ks_sink)(std::move(w));
    return;
  }
  const int nq = level + 1, nqp = nq + alpha;
  const u64 twoN = 2 * T.N;
  const int nblk = cdiv(T.N, TPB);
  const int rstep = std::min(MR_MAX, g_knobs.mr_rotations);
  const int mstep = std::min(MS_MAXB, g_knobs.mr_members);
  const int rpw = g_knobs.mr_group;
  for (int r0 = 0; r0 < nrot; r0 += rstep) {
    const int nr = std::min(nrot - r0, rstep);
    MultiRot R;
    R.accumulate = masks && accumulate ? 1 : 0;
    for (int r = 0; r < nr; r++) {
      R.out[r] = outs[r0 + r];
      R.key[r] = keys[r0 + r];
      R.mask[r] = masks ? masks[r0 + r] : nullptr;
      R.ginv[r] = inv_mod_2n(gs[r0 + r], twoN);
    }
    const PosList P = pos_order(T, nq, nqp, L);
    // the launch order split into FP64 and integer positions
    PosList pf, pi;
    int nf = 0, ni = 0;
    for (int x = 0; x < nqp; x++) {
      const int pos = P.pos[x];
      const int m = pos < nq ? pos : L + 1 + (pos - nq);
      if (T.bits[m] <= F64_LAZY_BITS) pf.pos[nf++] = (short)pos;
      else pi.pos[ni++] = (short)pos;
    }
    const bool split = ni > 0 && g_knobs.mr_int_split != 0;
    for (int b0 = 0; b0 < batch; b0 += mstep) {
      const int mb = batch - b0 < mstep ? batch - b0 : mstep;
      const MrCost all = mr_cost(T, P, nqp, nq, L, nr, mb, beta, c0 != nullptr, masks != nullptr, R.accumulate != 0);
      const MrCost fp = split ? mr_cost(T, pf, nf, nq, L, nr, mb, beta, c0 != nullptr, masks != nullptr,
                                        R.accumulate != 0)
                              : all;
      // FP64-only kernel when every launched limb is FP64 (the integer branch compiled out)
#define MR_LAUNCH(K, FP, G, PL, NP)                                                                                \
  hipLaunchKernelGGL((k_multsum_rot<K, FP, G>), dim3(cdiv(nblk, 8) * 8 * cdiv(nr, G), NP), dim3(TPB), 0, s, R, PL, \
                     nr, digits, c0, pmod, nq, nqp, L, beta, T.nmods, batch, b0, T.logN, T.mc)
#define MR_GROUPS(K, FP, PL, NP)             \
  if (rpw == 4) MR_LAUNCH(K, FP, 4, PL, NP); \
  else if (rpw == 2) MR_LAUNCH(K, FP, 2, PL, NP); \
  else MR_LAUNCH(K, FP, 1, PL, NP);
#define MR_CASE(K)                                     \
  case K:                                              \
    if (split) {                                       \
      MR_GROUPS(K, true, pf, nf)                       \
    } else if (ni) {                                   \
      MR_GROUPS(K, false, P, nqp)                      \
    } else {                                           \
      MR_GROUPS(K, true, P, nqp)                       \
    }                                                  \
    break;
      // the integer limbs' kernel first: on the forked stream it runs beside
      // the FP64 kernel, joined before anything else is launched on s
      const bool concurrent = split && fs && fs->aux && g_knobs.mr_int_concurrent != 0;
      if (split) {
        hipStream_t si = s;
        if (concurrent) {
          fork_check(hipEventRecord(fs->fork, s), "event record");
          fork_check(hipStreamWaitEvent(fs->aux, fs->fork, 0), "stream wait");
          si = fs->aux;
        }
        const MrCost ic = mr_cost(T, pi, ni, nq, L, nr, mb, beta, c0 != nullptr, masks != nullptr, R.accumulate != 0);
        ProfScope ps("multsum_rot_int", si, ic.bytes, ic.mm, ic.unit);
        const dim3 grid(cdiv(nblk, 8) * 8 * nr, ni);
        const int rc = std::min(nr, g_knobs.mr_int_chunk);
#define MRI_CASE(K)                                                                                              \
  case K:                                                                                                        \
    if (g_knobs.mr_int_pass == 8)                                                                                \
      hipLaunchKernelGGL((k_multsum_rot_int<K, 8>), grid, dim3(TPB), 0, si, R, pi, nr, rc, digits, c0, pmod, nq, \
                         nqp, L, beta, T.nmods, batch, b0, T.logN, T.mc);                                        \
    else                                                                                                         \
      hipLaunchKernelGGL((k_multsum_rot_int<K, 4>), grid, dim3(TPB), 0, si, R, pi, nr, rc, digits, c0, pmod, nq, \
                         nqp, L, beta, T.nmods, batch, b0, T.logN, T.mc);                                        \
    break;
        switch (mb) {
          MRI_CASE(1) MRI_CASE(2) MRI_CASE(3) MRI_CASE(4) MRI_CASE(5) MRI_CASE(6) MRI_CASE(7) MRI_CASE(8)
        }
#undef MRI_CASE
      }
      {
        // per member and rotation: 2 beta key products on every position, P c0
        // on the Q limbs, the mask on both halves
        ProfScope ps("multsum_rot", s, fp.bytes, fp.mm, fp.unit);
        switch (mb) {
          MR_CASE(1) MR_CASE(2) MR_CASE(3) MR_CASE(4) MR_CASE(5) MR_CASE(6) MR_CASE(7) MR_CASE(8)
        }
      }
      if (concurrent) {
        fork_check(hipEventRecord(fs->join, fs->aux), "event record");
        fork_check(hipStreamWaitEvent(s, fs->join, 0), "stream wait");
      }
    }
#undef MR_CASE
#undef MR_GROUPS
#undef MR_LAUNCH
  }
}
// Two bases under the same keys in one FP64 launch (the A side's two masked
// hoisted sums): outs[r] = masks[r] (rotation of base 1) + masks2[r]
// (rotation of base 2).  The 60-bit limbs run the two launches of their own
// kernel (the second accumulating).  False (nothing launched) where the pair
// launch does not apply: knob mr_pair off, a merged-launch sink, or 60-bit
// limbs that do not run in a kernel of their own.
bool launch_multsum_rot_pair(const DeviceTables& T, u64* const* outs, const u64* const* keys, const u64* gs, int nrot,
                             const u64* digits, const u64* c0, const u64* const* masks, const u64* digits2,
                             const u64* c02, const u64* const* masks2, const u64* pmod, int level, int L, int alpha,
                             int beta, int batch, hipStream_t s) {
  if (!g_knobs.mr_pair || tls_ks_sink || !masks || !masks2) return false;
  const int nq = level + 1, nqp = nq + alpha;
  const PosList P = pos_order(T, nq, nqp, L);
  PosList pf, pi;
  int nf = 0, ni = 0;
  for (int x = 0; x < nqp; x++) {
    const int pos = P.pos[x];
    const int m = pos < nq ? pos : L + 1 + (pos - nq);
    if (T.bits[m] <= F64_LAZY_BITS) pf.pos[nf++] = (short)pos;
    else pi.pos[ni++] = (short)pos;
  }
  if (ni > 0 && !g_knobs.mr_int_split) return false;
  const u64 twoN = 2 * T.N;
  const int nblk = cdiv(T.N, TPB);
  const int rstep = std::min(MR_MAX, g_knobs.mr_rotations);
  const int mstep = std::min(MS_MAXB, g_knobs.mr_members);
  constexpr int RPW = 2;  // 2 x 8 digit lanes: the sums of two rotations fill the registers
  for (int r0 = 0; r0 < nrot; r0 += rstep) {
    const int nr = std::min(nrot - r0, rstep);
    MultiRot R;
    R.accumulate = 0;
    R.digits2 = digits2;
    R.c02 = c02;
    for (int r = 0; r < nr; r++) {
      R.out[r] = outs[r0 + r];
      R.key[r] = keys[r0 + r];
      R.mask[r] = masks[r0 + r];
      R.mask2[r] = masks2[r0 + r];
      R.ginv[r] = inv_mod_2n(gs[r0 + r], twoN);
    }
    for (int b0 = 0; b0 < batch; b0 += mstep) {
      const int mb = batch - b0 < mstep ? batch - b0 : mstep;
      if (ni > 0) {
        // the 60-bit limbs: base 1, then base 2 added on
        MultiRot R2 = R;
        for (int r = 0; r < nr; r++) R2.mask[r] = masks2[r0 + r];
        R2.accumulate = 1;
        const dim3 grid(cdiv(nblk, 8) * 8 * nr, ni);
        const int rc = std::min(nr, g_knobs.mr_int_chunk);
        for (int half = 0; half < 2; half++) {
          const MultiRot& RI = half ? R2 : R;
          const MrCost ic = mr_cost(T, pi, ni, nq, L, nr, mb, beta, true, true, half == 1);
          ProfScope ps("multsum_rot_int", s, ic.bytes, ic.mm, ic.unit);
          const u64* dg = half ? digits2 : digits;
          const u64* cz = half ? c02 : c0;
#define MRP_INT(K)                                                                                                    \
  case K:                                                                                                             \
    if (g_knobs.mr_int_pass == 8)                                                                                     \
      hipLaunchKernelGGL((k_multsum_rot_int<K, 8>), grid, dim3(TPB), 0, s, RI, pi, nr, rc, dg, cz, pmod, nq, nqp, L, \
                         beta, T.nmods, batch, b0, T.logN, T.mc);                                                     \
    else                                                                                                              \
      hipLaunchKernelGGL((k_multsum_rot_int<K, 4>), grid, dim3(TPB), 0, s, RI, pi, nr, rc, dg, cz, pmod, nq, nqp, L, \
                         beta, T.nmods, batch, b0, T.logN, T.mc);                                                     \
    break;
          switch (mb) { MRP_INT(1) MRP_INT(2) MRP_INT(3) MRP_INT(4) MRP_INT(5) MRP_INT(6) MRP_INT(7) MRP_INT(8) }
#undef MRP_INT
        }
      }
      // the FP64 limbs: 2 mb digit lanes, each key word loaded once; the
      // outputs of mb members written once
      MrCost fp = mr_cost(T, pf, nf, nq, L, nr, 2 * mb, beta, true, true, false);
      fp.bytes -= 8.0 * T.N * nf * mb * nr * 2.0;
      ProfScope ps("multsum_rot", s, fp.bytes, fp.mm, fp.unit);
#define MRP_FP(K)                                                                                                    \
  case K:                                                                                                            \
    hipLaunchKernelGGL((k_multsum_rot<K, true, RPW, true>), dim3(cdiv(nblk, 8) * 8 * cdiv(nr, RPW), nf), dim3(TPB), \
                       0, s, R, pf, nr, digits, c0, pmod, nq, nqp, L, beta, T.nmods, batch, b0, T.logN, T.mc);      \
    break;
      switch (mb) { MRP_FP(1) MRP_FP(2) MRP_FP(3) MRP_FP(4) MRP_FP(5) MRP_FP(6) MRP_FP(7) MRP_FP(8) }
#undef MRP_FP
    }
  }
  return true;
}

void launch_multsum(const DeviceTables& T, u64* out, const u64* digits, const u64* key, const u64* c0,
                    const u64* pmod, int level, int L, int alpha, int beta, u64 g, int batch, hipStream_t s) {
  if (tls_ks_sink) {
    launch_multsum_rot(T, &out, &key, &g, 1, digits, c0, pmod, level, L, alpha, beta, batch, s);
    return;
  }
  int nq = level + 1, nqp = nq + alpha;
  dim3 grid(cdiv(T.N, TPB), nqp);
  const int mstep = std::min(MS_MAXB, g_knobs.ms_members);
  for (int b0 = 0; b0 < batch; b0 += mstep) {
    const int mb = batch - b0 < mstep ? batch - b0 : mstep;
    // key read once; digits and c0 of the mb members read once; outputs written once
    ProfScope ps("multsum", s, 8.0 * T.N * (2.0 * beta * nqp + mb * (beta * nqp + (c0 ? nq : 0) + 2.0 * nqp)),
                 mm_qp(T, nq, nqp, L, (double)T.N * (2.0 * beta + (c0 ? 1 : 0)), (double)T.N * 2.0 * beta, mb),
                 8.0 * T.N * (2.0 * beta * nqp + (double)mb * 4.0 * nq));
#define MS_CASE(K)                                                                                              \
  case K:                                                                                                       \
    hipLaunchKernelGGL(k_multsum<K>, grid, dim3(TPB), 0, s, out, digits, key, c0, pmod, nq, nqp, L, beta, T.nmods, \
                       batch, b0, g, T.logN, T.mc);                                                             \
    break;
    switch (mb) {
      MS_CASE(1) MS_CASE(2) MS_CASE(3) MS_CASE(4) MS_CASE(5) MS_CASE(6) MS_CASE(7) MS_CASE(8)
    }
#undef MS_CASE
  }
}

// P-lift of npoly polys [npoly][nq] -> [npoly][nqp]: P * c on Q limbs, 0 on P limbs
__global__ void k_plift(u64* out, const u64* c, const u64* pmod, int nq, int nqp, int logN,
                        const ModConst* __restrict__ mc) {
  const u64 N = 1ull << logN;
  u32 i = blockIdx.x * TPB + threadIdx.x;
  int pos = blockIdx.y, p = blockIdx.z;
  if (i >= N) return;
  u64 v = 0;
  if (pos < nq) v = mul_const_any(c[((size_t)p * nq + pos) * N + i], pmod[2 * pos], pmod[2 * pos + 1], mc[pos]);
  out[((size_t)p * nqp + pos) * N + i] = v;
}
void launch_plift(const DeviceTables& T, u64* out, const u64* c, const u64* pmod, int level, int alpha, int npoly,
                  hipStream_t s) {
  int nq = level + 1, nqp = nq + alpha;
  ProfScope ps("plift", s, 8.0 * T.N * npoly * ((double)nq + nqp), mm_q(T, nq, (double)T.N, npoly));
  dim3 grid(cdiv(T.N, TPB), nqp, npoly);
  hipLaunchKernelGGL(k_plift, grid, dim3(TPB), 0, s, out, c, pmod, nq, nqp, T.logN, T.mc);
}

// ---------------------------------------------------------------------------
// Rescale: t_i = [x_l]_{q_l} mod q_i (centred top limb), out_i = (x_i - t_i) q_l^{-1}
// ---------------------------------------------------------------------------
// t [npoly][nout][N] for the moduli q_0..q_{nout-1}, nout <= l
__global__ void k_rescale_lift(u64* t, const u64* top, int l, int nout, int logN, const ModConst* __restrict__ mc) {
  const u64 N = 1ull << logN;
  u32 i = blockIdx.x * TPB + threadIdx.x;
  int k = blockIdx.y, p = blockIdx.z;
  if (i >= N) return;
  u64 ql = mc[l].q;
  u64 x = top[(size_t)p * N + i];
  const ModConst mk = mc[k];
  u64 v;
  if (x > (ql >> 1)) {
    u64 r = reduce64(ql - x, mk);
    v = r ? mk.q - r : 0;
  } else {
    v = reduce64(x, mk);
  }
  t[((size_t)p * nout + k) * N + i] = v;
}
void launch_rescale_lift(const DeviceTables& T, u64* t, const u64* top_coef, int l, int nout, int npoly,
                         hipStream_t s) {
  ProfScope ps("rescale_lift", s, 8.0 * T.N * npoly * (1.0 + nout));
  dim3 grid(cdiv(T.N, TPB), nout, npoly);
  hipLaunchKernelGGL(k_rescale_lift, grid, dim3(TPB), 0, s, t, top_coef, l, nout, T.logN, T.mc);
}
__global__ void k_rescale_final(u64* out, const u64* x, const u64* t, int l, int x_stride_limbs, const u64* qlinv,
                                int logN, const ModConst* __restrict__ mc) {
  const u64 N = 1ull << logN;
  u32 i = blockIdx.x * TPB + threadIdx.x;
  int k = blockIdx.y, p = blockIdx.z;
  if (i >= N) return;
  u64 q = mc[k].q;
  u64 d = sub_mod(x[((size_t)p * x_stride_limbs + k) * N + i], t[((size_t)p * l + k) * N + i], q);
  out[((size_t)p * l + k) * N + i] = mul_const_any(d, qlinv[2 * k], qlinv[2 * k + 1], mc[k]);
}
void launch_rescale_final(const DeviceTables& T, u64* out, const u64* x, const u64* t, int l, int npoly,
                          int x_stride_limbs, const u64* qlinv, hipStream_t s) {
  ProfScope ps("rescale_final", s, 8.0 * T.N * npoly * 3.0 * l, mm_q(T, l, (double)T.N, npoly));
  dim3 grid(cdiv(T.N, TPB), l, npoly);
  hipLaunchKernelGGL(k_rescale_final, grid, dim3(TPB), 0, s, out, x, t, l, x_stride_limbs, qlinv, T.logN, T.mc);
}

// Rescale with the lift fused into the forward column pass: the value of
// limb k at a coefficient is the centred top-limb residue reduced mod q_k,
// computed while filling the tile; the block pass ends with (x - t) q_l^-1.
struct LiftLoad {
  typedef u64 Raw;
  const u64* top;
  u64 ql;
  ModConst mk;
  __device__ __forceinline__ void raw(size_t idx, Raw& r) const { r = top[idx]; }
  __device__ __forceinline__ u64 fin_u(const Raw& x) const {
    if (x > (ql >> 1)) {
      const u64 r = reduce64(ql - x, mk);
      return r ? mk.q - r : 0;
    }
    return reduce64(x, mk);
  }
};
// top limb and target both below 2^46: centred top residue reduced in FP64
struct LiftLoadF64 {
  typedef u64 Raw;
  const u64* top;
  double ql, q, qinv;
  __device__ __forceinline__ void raw(size_t idx, Raw& r) const { r = top[idx]; }
  __device__ __forceinline__ double fin_d(const Raw& r) const {
    const double x = u2d(r);
    return f64_centre(x > 0.5 * ql ? x - ql : x, q, qinv);
  }
  __device__ __forceinline__ u64 fin_u(const Raw& r) const { return d2u(f64_canon(fin_d(r), q, qinv)); }
};
__device__ __forceinline__ double fin(const F64LazyArith&, const LiftLoadF64& ld, const u64& r) { return ld.fin_d(r); }
template <int LOGN, int GA, int GB>
__global__ void __launch_bounds__(TPB) k_ntt_cols2_lift(u64* t, const u64* __restrict__ top, int l, int nout,
                                                        const u64* __restrict__ tw, const u64* __restrict__ twsh,
                                                        const double* __restrict__ twf,
                                                        const ModConst* __restrict__ mc) {
  constexpr int S1 = GA + GB, R = 1 << S1, C = TILE / R;
  __shared__ u64 sh[LDS_WORDS];
  const int limb = blockIdx.y;
  const int p = limb / nout, k = limb - p * nout;
  const u64 N = 1ull << LOGN;
  u64* a = t + (size_t)limb * N;
  const int c0 = blockIdx.x * C;
  const ModConst mk = mc[k];
  LiftLoad ld{top + (size_t)p * N, mc[l].q, mk};
  if (mk.bits <= F64_LAZY_BITS) {
    F64LazyArith ar{twf + (size_t)k * N, mk.qf, mk.qinvf, (double)mk.ninv};
    if (mc[l].bits <= F64_LAZY_BITS)
      ntt_cols2_body<LOGN, GA, GB, false>(a, c0, reinterpret_cast<double*>(sh), ar,
                                          LiftLoadF64{top + (size_t)p * N, mc[l].qf, mk.qf, mk.qinvf});
    else
      ntt_cols2_body<LOGN, GA, GB, false>(a, c0, reinterpret_cast<double*>(sh), ar, ld);
  } else {
    ShoupArith ar{tw + (size_t)k * N, twsh + (size_t)k * N, mk.q, mk.ninv, mk.ninv_sh};
    ntt_cols2_body<LOGN, GA, GB, false>(a, c0, sh, ar, ld);
  }
}
template <int LOGN, int GA, int GB, int GC, int GD>
static void rescale_fused(const DeviceTables& T, u64* t, const u64* top, int l, int nout, int npoly, const u64* x,
                          int x_stride, const u64* cpairs, u64* out, hipStream_t s) {
  constexpr int R = 1 << (GA + GB), C = TILE / R;
  dim3 gc((1 << LOGN) / R / C, nout * npoly);
  {
    ProfScope ps("ntt_fwd_cols_lift", s, 8.0 * T.N * npoly * (1.0 + nout), mm_q(T, nout, 0.5 * T.N * (GA + GB), npoly));
    hipLaunchKernelGGL((k_ntt_cols2_lift<LOGN, GA, GB>), gc, dim3(TPB), 0, s, t, top, l, nout, T.psi, T.psi_sh,
                       T.psi_f, T.mc);
  }
  LimbMap map;
  map.n = nout;
  for (int k = 0; k < nout; k++) map.idx[k] = (short)k;
  ntt2_fwd_sub<LOGN, GA, GB, GC, GD>(T, t, nout, npoly, map, x, x_stride, cpairs, out, s, false);
}
bool launch_rescale_fused(const DeviceTables& T, u64* t, const u64* top_coef, int l, int nout, int npoly,
                          const u64* x, int x_stride, const u64* cpairs, u64* out, hipStream_t s) {
  return ntt_dispatch(T.logN, [&](auto sp) {
    using S = decltype(sp);
    rescale_fused<NTT_SPLIT_ARGS>(T, t, top_coef, l, nout, npoly, x, x_stride, cpairs, out, s);
  });
}

// ---------------------------------------------------------------------------
// Philox4x64-10 (Salmon et al., SC'11) and the samplers
// ---------------------------------------------------------------------------
__device__ __forceinline__ void philox4x64(u64 c[4], u64 k0, u64 k1) {
  const u64 M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
  const u64 W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
#pragma unroll
  for (int r = 0; r < 10; r++) {
    if (r) { k0 += W0; k1 += W1; }
    u64 hi0 = mulhi64(M0, c[0]), lo0 = M0 * c[0];
    u64 hi1 = mulhi64(M1, c[2]), lo1 = M1 * c[2];
    u64 n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
    c[0] = n0; c[1] = lo1; c[2] = n2; c[3] = lo0;
  }
}

// uniform residues drawn directly in the evaluation domain:
// counter (i, modulus index, c2, c3); value (w0 2^64 + w1) mod q
__global__ void k_sample_uniform(u64* out, int nlimbs, LimbMap map, u64 seed, u64 tag, u64 c2, u64 c3, int logN,
                                 const ModConst* __restrict__ mc) {
  const u64 N = 1ull << logN;
  u32 i = blockIdx.x * TPB + threadIdx.x;
  int k = blockIdx.y;
  if (i >= N) return;
  int m = limb_mod(map, k);
  if (m < 0) return;
  u64 c[4] = {i, (u64)m, c2, c3};
  philox4x64(c, seed, tag);
  const ModConst mk = mc[m];
  u64 hi = reduce64(c[0], mk);
  u64 v = add_mod(shoup_mul(hi, mk.r64, mk.r64_sh, mk.q), reduce64(c[1], mk), mk.q);
  out[(size_t)k * N + i] = v;
}
void launch_sample_uniform(const DeviceTables& T, u64* out, int nlimbs, const LimbMap& m, u64 seed, u64 tag, u64 c2,
                           u64 c3, hipStream_t s) {
  dim3 grid(cdiv(T.N, TPB), nlimbs);
  hipLaunchKernelGGL(k_sample_uniform, grid, dim3(TPB), 0, s, out, nlimbs, m, seed, tag, c2, c3, T.logN, T.mc);
}

__global__ void k_sample_small(i64* out, int kind, u64 seed, u64 tag, u64 c1, u64 c2, u64 c3, int logN,
                               const u64* __restrict__ cdt) {
  const u64 N = 1ull << logN;
  u32 i = blockIdx.x * TPB + threadIdx.x;
  if (i >= N) return;
  u64 c[4] = {i, c1, c2, c3};
  philox4x64(c, seed, tag);
  i64 v;
  if (kind == 0) {
    v = (i64)(c[0] % 3) - 1;
  } else {
    v = -19;
    for (int k = 0; k < 38; k++) v += c[0] >= cdt[k] ? 1 : 0;
  }
  out[i] = v;
}
void launch_sample_ternary(const DeviceTables& T, i64* out, u64 seed, u64 tag, u64 c1, u64 c2, u64 c3,
                           hipStream_t s) {
  hipLaunchKernelGGL(k_sample_small, dim3(cdiv(T.N, TPB)), dim3(TPB), 0, s, out, 0, seed, tag, c1, c2, c3, T.logN,
                     T.cdt);
}
void launch_sample_gauss(const DeviceTables& T, i64* out, u64 seed, u64 tag, u64 c1, u64 c2, u64 c3,
                         hipStream_t s) {
  hipLaunchKernelGGL(k_sample_small, dim3(cdiv(T.N, TPB)), dim3(TPB), 0, s, out, 1, seed, tag, c1, c2, c3, T.logN,
                     T.cdt);
}
__global__ void k_add_int(i64* out, const i64* a, const i64* b, u64 N) {
  u64 i = (u64)blockIdx.x * TPB + threadIdx.x;
  if (i < N) out[i] = a[i] + b[i];
}
void launch_add_int(i64* out, const i64* a, const i64* b, u64 N, hipStream_t s) {
  hipLaunchKernelGGL(k_add_int, dim3(cdiv(N, TPB)), dim3(TPB), 0, s, out, a, b, N);
}

// m <- round(m * mant / 2^shift), halves away from zero, exact (128-bit product)
__global__ void k_scale_int(i64* m, u64 mant, int shift, u64 N) {
  u64 i = (u64)blockIdx.x * TPB + threadIdx.x;
  if (i >= N) return;
  i64 v = m[i];
  u64 a = v < 0 ? (u64)0 - (u64)v : (u64)v;
  u64 lo = a * mant, hi = mulhi64(a, mant);
  // + 2^(shift-1)
  if (shift - 1 < 64) {
    u64 add = 1ull << (shift - 1);
    u64 l2 = lo + add;
    hi += l2 < lo;
    lo = l2;
  } else {
    hi += 1ull << (shift - 1 - 64);
  }
  u64 r = shift < 64 ? (lo >> shift) | (hi << (64 - shift)) : hi >> (shift - 64);
  m[i] = v < 0 ? -(i64)r : (i64)r;
}
void launch_scale_int(i64* m, u64 mant, int shift, u64 N, hipStream_t s) {
  hipLaunchKernelGGL(k_scale_int, dim3(cdiv(N, TPB)), dim3(TPB), 0, s, m, mant, shift, N);
}

// b = e - a s (+ (P mod q) s' on the primes of digit `digit`)
__global__ void k_swk_b(u64* b, const u64* a, const u64* e, const u64* s_ntt, const u64* sp_ntt, const u64* pmod,
                        int digit, int alpha, int L, int logN, const ModConst* __restrict__ mc) {
  const u64 N = 1ull << logN;
  u32 i = blockIdx.x * TPB + threadIdx.x;
  int m = blockIdx.y;
  if (i >= N) return;
  const ModConst mk = mc[m];
  size_t o = (size_t)m * N + i;
  u64 v = sub_mod(e[o], mul_mod(a[o], s_ntt[o], mk), mk.q);
  if (sp_ntt && m <= L && m / alpha == digit) v = add_mod(v, mul_mod(pmod[2 * m], sp_ntt[o], mk), mk.q);
  b[o] = v;
}
void launch_swk_b(const DeviceTables& T, u64* b, const u64* a, const u64* e, const u64* s_ntt, const u64* sp_ntt,
                  const u64* pmod, int nlimbs_total, int digit, int alpha, int L, hipStream_t s) {
  dim3 grid(cdiv(T.N, TPB), nlimbs_total);
  hipLaunchKernelGGL(k_swk_b, grid, dim3(TPB), 0, s, b, a, e, s_ntt, sp_ntt, pmod, digit, alpha, L, T.logN, T.mc);
}

// A switching key's limbs of at most F64_LAZY_BITS bits rewritten in place as
// the IEEE doubles of their residues (exact below 2^53): the key inner
// products read them as FP64 operands with no conversion.  The 60-bit limbs
// stay integers.
__global__ void k_key_f64(u64* key, int nmods, int logN, const ModConst* __restrict__ mc) {
  const u64 N = 1ull << logN;
  const u32 i = blockIdx.x * TPB + threadIdx.x;
  const int m = (int)blockIdx.y % nmods;
  if (i >= N || mc[m].bits > F64_LAZY_BITS) return;
  u64* p = key + (size_t)blockIdx.y * N + i;
  *p = (u64)__double_as_longlong((double)*p);
}
void launch_key_f64(const DeviceTables& T, u64* key, int nblocks, int nmods, hipStream_t s) {
  dim3 grid(cdiv(T.N, TPB), nblocks * nmods);
  hipLaunchKernelGGL(k_key_f64, grid, dim3(TPB), 0, s, key, nmods, T.logN, T.mc);
}

// centred integer of one coefficient-domain limb
__global__ void k_centre(i64* out, const u64* coef, int m, int logN, const ModConst* __restrict__ mc) {
  const u64 N = 1ull << logN;
  u32 i = blockIdx.x * TPB + threadIdx.x;
  if (i >= N) return;
  u64 q = mc[m].q, x = coef[i];
  out[i] = x > (q >> 1) ? -(i64)(q - x) : (i64)x;
}
void launch_centre_to_int(const DeviceTables& T, i64* out, const u64* coef, int mod, hipStream_t s) {
  hipLaunchKernelGGL(k_centre, dim3(cdiv(T.N, TPB)), dim3(TPB), 0, s, out, coef, mod, T.logN, T.mc);
}

// ---------------------------------------------------------------------------
// Canonical embedding in double-double arithmetic (Dekker / Knuth error-free
// transformations).  Encoding computes
//   v_i = (Delta / N) Re( zeta^-i sum_t u[t] w^(-t i) ),   m_i = floor(v_i + 1/2 + 2^-30)
// with u[t] = z_j at the odd exponents 2t+1 = +-5^j mod 2N.
// ---------------------------------------------------------------------------
struct dd { double hi, lo; };
struct cdd { dd re, im; };

__device__ __forceinline__ dd two_sum(double a, double b) {
  double s = a + b, bb = s - a;
  return {s, (a - (s - bb)) + (b - bb)};
}
__device__ __forceinline__ dd quick_two_sum(double a, double b) {
  double s = a + b;
  return {s, b - (s - a)};
}
__device__ __forceinline__ dd dd_add(dd a, dd b) {
  dd s = two_sum(a.hi, b.hi), t = two_sum(a.lo, b.lo);
  s.lo += t.hi;
  s = quick_two_sum(s.hi, s.lo);
  s.lo += t.lo;
  return quick_two_sum(s.hi, s.lo);
}
__device__ __forceinline__ dd dd_neg(dd a) { return {-a.hi, -a.lo}; }
__device__ __forceinline__ dd dd_mul(dd a, dd b) {
  double p = a.hi * b.hi;
  double e = fma(a.hi, b.hi, -p);
  e += a.hi * b.lo + a.lo * b.hi;
  return quick_two_sum(p, e);
}
__device__ __forceinline__ dd dd_mul_d(dd a, double b) {
  double p = a.hi * b;
  double e = fma(a.hi, b, -p);
  e += a.lo * b;
  return quick_two_sum(p, e);
}
__device__ __forceinline__ cdd cdd_mul(cdd a, cdd b) {
  return {dd_add(dd_mul(a.re, b.re), dd_neg(dd_mul(a.im, b.im))), dd_add(dd_mul(a.re, b.im), dd_mul(a.im, b.re))};
}
__device__ __forceinline__ cdd cdd_add(cdd a, cdd b) { return {dd_add(a.re, b.re), dd_add(a.im, b.im)}; }
__device__ __forceinline__ cdd cdd_sub(cdd a, cdd b) { return {dd_add(a.re, dd_neg(b.re)), dd_add(a.im, dd_neg(b.im))}; }

// scatter the message into bit-reversed FFT input order
__global__ void k_enc_scatter(cdd* x, const double* z, int nz, int batch, int logN, const u32* rotgroup) {
  const u64 N = 1ull << logN, S = N >> 1;
  u64 j = (u64)blockIdx.x * TPB + threadIdx.x;
  int b = blockIdx.y;
  if (j >= S) return;
  double v = z[(size_t)b * nz + (j % nz)];
  u32 e = rotgroup[j];
  u32 t1 = (e - 1) >> 1, t2 = (u32)((2 * N - e - 1) >> 1);
  cdd val = {{v, 0.0}, {0.0, 0.0}};
  x[(size_t)b * N + brv(t1, logN)] = val;
  x[(size_t)b * N + brv(t2, logN)] = val;
}

// one radix-2 stage of an in-place DIT FFT (input in bit-reversed order);
// sign = -1 uses exp(-2 pi i k/N), +1 its conjugate
__global__ void k_fft_stage(cdd* x, int logN, int len, int sign, const double* tw) {
  const u64 N = 1ull << logN;
  u64 t = (u64)blockIdx.x * TPB + threadIdx.x;
  int b = blockIdx.y;
  if (t >= N / 2) return;
  int half = len >> 1;
  u64 blk = t / half, k = t % half;
  u64 i0 = blk * len + k, i1 = i0 + half;
  u64 ti = k * (N / len);
  const double* w4 = tw + 4 * ti;
  cdd w = {{w4[0], w4[1]}, {sign < 0 ? w4[2] : -w4[2], sign < 0 ? w4[3] : -w4[3]}};
  cdd* xb = x + (size_t)b * N;
  cdd a = xb[i0], c = cdd_mul(xb[i1], w);
  xb[i0] = cdd_add(a, c);
  xb[i1] = cdd_sub(a, c);
}

__global__ void k_enc_finish(i64* out, const cdd* x, double delta_over_n, int logN, const double* zeta) {
  const u64 N = 1ull << logN;
  u64 i = (u64)blockIdx.x * TPB + threadIdx.x;
  int b = blockIdx.y;
  if (i >= N) return;
  cdd U = x[(size_t)b * N + i];
  dd c = {zeta[4 * i], zeta[4 * i + 1]}, s = {zeta[4 * i + 2], zeta[4 * i + 3]};
  // Re(zeta^-i U) = Re(U) cos + Im(U) sin
  dd re = dd_add(dd_mul(U.re, c), dd_mul(U.im, s));
  dd v = dd_mul_d(re, delta_over_n);
  dd w = dd_add(v, dd{0.500000000931322574615478515625, 0.0});  // 1/2 + 2^-30, exact
  double f = floor(w.hi);
  i64 r = (i64)f;
  if (f == w.hi && w.lo < 0.0) r -= 1;
  out[(size_t)b * N + i] = r;
}

size_t encode_scratch_bytes(const DeviceTables& T, int batch) { return (size_t)batch * T.N * sizeof(cdd); }

void launch_encode(const DeviceTables& T, i64* out, const double* z, int nz, int batch, double delta, void* scratch,
                   hipStream_t s) {
  cdd* x = (cdd*)scratch;  // every entry is written by the scatter (+-5^j cover all odd residues)
  hipLaunchKernelGGL(k_enc_scatter, dim3(cdiv(T.N / 2, TPB), batch), dim3(TPB), 0, s, x, z, nz, batch, T.logN,
                     T.rotgroup);
  for (int len = 2; len <= (int)T.N; len <<= 1)
    hipLaunchKernelGGL(k_fft_stage, dim3(cdiv(T.N / 2, TPB), batch), dim3(TPB), 0, s, x, T.logN, len, -1, T.fft_tw);
  hipLaunchKernelGGL(k_enc_finish, dim3(cdiv(T.N, TPB), batch), dim3(TPB), 0, s, out, x, delta / (double)T.N,
                     T.logN, T.zeta);
}

// decoding: y[t] = sum_i (m_i zeta^i) w^(t i); z_j = Re(y[(5^j - 1)/2]) / scale
__global__ void k_dec_scatter(cdd* x, const i64* m, int logN, const double* zeta) {
  const u64 N = 1ull << logN;
  u64 i = (u64)blockIdx.x * TPB + threadIdx.x;
  int b = blockIdx.y;
  if (i >= N) return;
  i64 v = m[(size_t)b * N + i];
  double hi = (double)v;
  double lo = (double)(v - (i64)hi);
  dd mv = quick_two_sum(hi, lo);
  dd c = {zeta[4 * i], zeta[4 * i + 1]}, s = {zeta[4 * i + 2], zeta[4 * i + 3]};
  x[(size_t)b * N + brv((u32)i, logN)] = {dd_mul(mv, c), dd_mul(mv, s)};
}
__global__ void k_dec_gather(double* out, const cdd* x, int logN, const u32* rotgroup, const double* inv_scale) {
  const u64 N = 1ull << logN, S = N >> 1;
  u64 j = (u64)blockIdx.x * TPB + threadIdx.x;
  int b = blockIdx.y;
  if (j >= S) return;
  cdd y = x[(size_t)b * N + ((rotgroup[j] - 1) >> 1)];
  out[(size_t)b * S + j] = (y.re.hi + y.re.lo) * inv_scale[b];
}
void launch_decode(const DeviceTables& T, double* out, const i64* m, int batch, const double* inv_scale,
                   void* scratch, hipStream_t s) {
  cdd* x = (cdd*)scratch;
  hipLaunchKernelGGL(k_dec_scatter, dim3(cdiv(T.N, TPB), batch), dim3(TPB), 0, s, x, m, T.logN, T.zeta);
  for (int len = 2; len <= (int)T.N; len <<= 1)
    hipLaunchKernelGGL(k_fft_stage, dim3(cdiv(T.N / 2, TPB), batch), dim3(TPB), 0, s, x, T.logN, len, +1, T.fft_tw);
  hipLaunchKernelGGL(k_dec_gather, dim3(cdiv(T.N / 2, TPB), batch), dim3(TPB), 0, s, out, x, T.logN, T.rotgroup,
                     inv_scale);
}
