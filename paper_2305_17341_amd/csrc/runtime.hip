// Host runtime of the MI355X RNS-CKKS library: parameters and tables, device
// memory, key generation, the CKKS operations, the double-hoisted linear
// transforms and Jiang's matrix product.  The C ABI wrappers live in abi.hip.
#include <cstring>

#include "runtime.h"

#include <algorithm>
#include <cmath>
#include <condition_variable>
#include <exception>
#include <mutex>
#include <thread>
#include <cstdio>
#include <set>
#include <unordered_map>

extern "C" void he_host_dd_tables(int logN, double* fft_tw, double* zeta);

typedef unsigned __int128 u128;

thread_local std::string g_last_error;

void hip_check(hipError_t e, const char* what) {
  if (e != hipSuccess) fail(HE_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

// ---------------------------------------------------------------------------
// device memory pool
// ---------------------------------------------------------------------------
void* DevPool::get(size_t bytes) {
  if (redirect) return redirect->get(bytes);
  if (bytes == 0) bytes = 8;
  bytes = (bytes + 255) & ~(size_t)255;
  if (bump_base) {
    if (bytes > bump_cap - bump_off) fail(HE_ENOMEM, "allocation-free workspace exhausted");
    void* p = bump_base + bump_off;
    bump_off += bytes;
    peak = std::max(peak, bump_off);
    return p;
  }
  auto it = free_.lower_bound(bytes);
  if (it != free_.end() && it->first <= (exact ? bytes : bytes + bytes / 4)) {
    void* p = it->second;
    size_t sz = it->first;
    free_.erase(it);
    bytes_cached -= sz;
    live_[p] = sz;
    bytes_live += sz;
    peak = std::max(peak, bytes_live);
    return p;
  }
  if (frozen) fail(HE_ENOMEM, "graph arena exhausted while recording");
  void* p = nullptr;
  for (int attempt = 0; attempt < 2; attempt++) {
    if (user_alloc) {
      p = user_alloc(bytes, user);
    } else if (hipMalloc(&p, bytes) != hipSuccess) {
      (void)hipGetLastError();
      p = nullptr;
    }
    if (p) break;
    trim();
  }
  if (!p) fail(HE_ENOMEM, "device allocation of " + std::to_string(bytes) + " bytes failed");
  live_[p] = bytes;
  bytes_live += bytes;
  peak = std::max(peak, bytes_live);
  return p;
}
void DevPool::put(void* p) {
  if (redirect && redirect->live_.count(p)) {
    redirect->put(p);
    return;
  }
  auto it = live_.find(p);
  if (it == live_.end()) return;
  size_t sz = it->second;
  live_.erase(it);
  bytes_live -= sz;
  free_.insert({sz, p});
  bytes_cached += sz;
}
void DevPool::wait() {
  if (stream) (void)hipStreamSynchronize(stream);
  else (void)hipDeviceSynchronize();
}
void DevPool::trim() {
  if (free_.empty()) return;
  wait();
  for (auto& kv : free_) {
    if (user_release) user_release(kv.second, user);
    else (void)hipFree(kv.second);
  }
  free_.clear();
  bytes_cached = 0;
}
DevPool::~DevPool() {
  if (free_.empty() && live_.empty()) return;
  wait();
  trim();
  for (auto& kv : live_) {
    if (user_release) user_release(kv.first, user);
    else (void)hipFree(kv.first);
  }
}

// ---------------------------------------------------------------------------
// host number theory
// ---------------------------------------------------------------------------
static u64 hmul(u64 a, u64 b, u64 q) { return (u64)((u128)a * b % q); }
static u64 hpow(u64 b, u64 e, u64 q) {
  u64 r = 1 % q;
  b %= q;
  for (; e; e >>= 1) {
    if (e & 1) r = hmul(r, b, q);
    b = hmul(b, b, q);
  }
  return r;
}
static u64 hinv(u64 a, u64 q) { return hpow(a % q, q - 2, q); }
u64 shoup_pre(u64 w, u64 q) { return (u64)(((u128)w << 64) / q); }

// Primality below 2^64: strong-probable-prime tests to the seven bases of
// Sinclair's set, which no composite below 2^64 passes.
static bool is_prime_u64(u64 n) {
  if (n < 2) return false;
  for (u64 p : {2ull, 3ull, 5ull, 7ull, 11ull, 13ull})
    if (n % p == 0) return n == p;
  const int s = __builtin_ctzll(n - 1);
  const u64 d = (n - 1) >> s;
  for (u64 base : {2ull, 325ull, 9375ull, 28178ull, 450775ull, 9780504ull, 1795265022ull}) {
    const u64 a = base % n;
    if (a == 0) continue;
    u64 x = hpow(a, d, n);
    if (x == 1 || x == n - 1) continue;
    bool witness = true;
    for (int r = 1; r < s; r++) {
      x = hmul(x, x, n);
      if (x == n - 1) {
        witness = false;
        break;
      }
    }
    if (witness) return false;
  }
  return true;
}

// Jacobi symbol (a / n) for odd n > 0 (binary method)
static int jacobi(u64 a, u64 n) {
  int t = 1;
  a %= n;
  while (a) {
    const int z = __builtin_ctzll(a);
    a >>= z;
    if ((z & 1) && ((n & 7) == 3 || (n & 7) == 5)) t = -t;
    if ((a & 3) == 3 && (n & 3) == 3) t = -t;
    std::swap(a, n);
    a %= n;
  }
  return n == 1 ? t : 0;
}

static u32 brv_host(u32 x, int bits) {
  u32 r = 0;
  for (int i = 0; i < bits; i++) r |= ((x >> i) & 1u) << (bits - 1 - i);
  return r;
}

// ---------------------------------------------------------------------------
// context construction
// ---------------------------------------------------------------------------
HeCtxImpl::~HeCtxImpl() {
  if (stream) (void)hipStreamSynchronize(stream);
  graphs.clear();
  ltplans.clear();
  ptcache.clear();
  keys.clear();
  s_ntt.release();
  pk.release();
  tables.clear();
  for (auto& row : up)
    for (auto& t : row) (void)t;
  if (ev0) (void)hipEventDestroy(ev0);
  if (ev1) (void)hipEventDestroy(ev1);
  // the pool is destroyed after this body: its last trim must not wait on a
  // stream that is gone (or, for a caller's stream, may be gone)
  pool.stream = nullptr;
  if (fork.aux) (void)hipStreamSynchronize(fork.aux);
  if (fork.fork) (void)hipEventDestroy(fork.fork);
  if (fork.join) (void)hipEventDestroy(fork.join);
  if (fork.aux) (void)hipStreamDestroy(fork.aux);
  if (own_stream && stream) (void)hipStreamDestroy(stream);
}

LimbMap HeCtxImpl::qmap(int nq) const {
  LimbMap m;
  m.n = nq;
  for (int k = 0; k < nq; k++) m.idx[k] = (short)k;
  return m;
}
LimbMap HeCtxImpl::qpmap(int level) const {
  LimbMap m;
  m.n = nqp_of(level);
  for (int k = 0; k < m.n; k++) m.idx[k] = (short)qp_mod(level, k);
  return m;
}
LimbMap HeCtxImpl::one(int mod) const {
  LimbMap m;
  m.n = 1;
  m.idx[0] = (short)mod;
  return m;
}
u64 HeCtxImpl::galois(long step) const {
  long S = (long)(N / 2);
  u64 r = (u64)(((step % S) + S) % S);
  u64 g = 1, b = 5;
  for (; r; r >>= 1, b = (b * b) % (2 * N))   // 5^r mod 2N, 2N <= 2^17
    if (r & 1) g = (g * b) % (2 * N);
  return g;
}
u64* HeCtxImpl::table_upload(const void* host, size_t bytes) {
  tables.emplace_back(&pool, (bytes + 7) / 8);
  hip_check(hipMemcpy(tables.back().p, host, bytes, hipMemcpyHostToDevice), "table upload");
  return tables.back().p;
}

// Setparams (Appendix A): every modulus is 1 mod 2N.  For each bit size b the
// largest such primes below 2^b are used, Q's in chain order first, then P's.
// 2^b is a multiple of 2N here (b >= 30 > log2 2N), so the candidates below
// it are 2^b - 2N + 1, 2^b - 4N + 1, ...; a size's next search starts below
// the prime it last gave.
static void choose_primes(int logN, const std::vector<int>& bits, u64* out) {
  const u64 step = 2ull << logN;
  std::map<int, u64> below;  // bit size -> the last prime taken of that size
  for (size_t k = 0; k < bits.size(); k++) {
    const int b = bits[k];
    const u64 lowest = 1ull << (b - 1);
    u64 q = below.count(b) ? below[b] - step : (1ull << b) - step + 1;
    while (q > lowest && !is_prime_u64(q)) q -= step;
    if (q <= lowest) fail(HE_EINVAL, "not enough NTT-friendly primes of this size");
    out[k] = q;
    below[b] = q;
  }
}

// psi of Appendix A's NTT: x^((q-1)/2N) has order exactly 2N iff its N-th
// power is -1, i.e. iff x^((q-1)/2) = -1: x is a quadratic non-residue
// (Euler's criterion).  The smallest non-residue x >= 2 is found with the
// Jacobi symbol.
static u64 root_2n(u64 q, int logN) {
  u64 x = 2;
  while (jacobi(x, q) != -1) x++;
  return hpow(x, (q - 1) >> (logN + 1), q);
}

// host-only: the moduli and NTT roots a context with these prime sizes uses
void params_moduli(int logN, const std::vector<int>& bits, u64* moduli, u64* psi) {
  choose_primes(logN, bits, moduli);
  for (size_t k = 0; k < bits.size(); k++) psi[k] = root_2n(moduli[k], logN);
}

static FbcTable make_fbc(HeCtxImpl* c, const std::vector<int>& src) {
  FbcTable t;
  t.ns = (int)src.size();
  std::vector<u64> hat((size_t)t.ns * c->nmods), hat_sh((size_t)t.ns * c->nmods);
  for (int a = 0; a < t.ns; a++) {
    t.src[a] = src[a];
    u64 qa = c->mods[src[a]];
    u64 h = 1;
    for (int b = 0; b < t.ns; b++)
      if (b != a) h = hmul(h, c->mods[src[b]] % qa, qa);
    t.hatinv[a] = hinv(h, qa);
    t.hatinv_sh[a] = shoup_pre(t.hatinv[a], qa);
    for (int m = 0; m < c->nmods; m++) {
      u64 qt = c->mods[m], ht = 1;
      for (int b = 0; b < t.ns; b++)
        if (b != a) ht = hmul(ht, c->mods[src[b]] % qt, qt);
      hat[(size_t)a * c->nmods + m] = ht;
      hat_sh[(size_t)a * c->nmods + m] = shoup_pre(ht, qt);
    }
  }
  t.hat_t = c->table_upload(hat.data(), hat.size() * 8);
  t.hat_t_sh = c->table_upload(hat_sh.data(), hat_sh.size() * 8);
  // D and its cofactors as 4-word integers (for the exact centred lift)
  auto mul_words = [](u64* w, u64 v) {
    u128 carry = 0;
    for (int k = 0; k < 4; k++) {
      u128 p = (u128)w[k] * v + carry;
      w[k] = (u64)p;
      carry = p >> 64;
    }
  };
  for (int k = 0; k < 4; k++) t.Dw[k] = 0;
  t.Dw[0] = 1;
  for (int a = 0; a < t.ns; a++) mul_words(t.Dw, c->mods[src[a]]);
  for (int a = 0; a < t.ns; a++) {
    for (int k = 0; k < 4; k++) t.Hw[a][k] = 0;
    t.Hw[a][0] = 1;
    for (int b = 0; b < t.ns; b++)
      if (b != a) mul_words(t.Hw[a], c->mods[src[b]]);
    t.qd[a] = (double)c->mods[src[a]];
  }
  std::vector<u64> dm((size_t)c->nmods * 2);
  for (int m = 0; m < c->nmods; m++) {
    u64 qt = c->mods[m], d = 1;
    for (int a = 0; a < t.ns; a++) d = hmul(d, c->mods[src[a]] % qt, qt);
    dm[2 * m] = d;
    dm[2 * m + 1] = shoup_pre(d, qt);
  }
  t.D_mod_t = c->table_upload(dm.data(), dm.size() * 8);
  // FP64 form for targets of 33 to 46 bits: a source value v (any size below 2^64)
  // is split v = v_hi 2^32 + v_lo, and v hat = v_lo hat + v_hi (2^32 hat) mod
  // q_t, both factors below q_t: [a][t] = (hat mod q_t, 2^32 hat mod q_t, D mod q_t)
  std::vector<double> hf((size_t)t.ns * c->nmods * 3);
  for (int a = 0; a < t.ns; a++)
    for (int m = 0; m < c->nmods; m++) {
      u64 qt = c->mods[m], h = hat[(size_t)a * c->nmods + m];
      double* e = &hf[((size_t)a * c->nmods + m) * 3];
      e[0] = (double)h;
      e[1] = (double)hmul(h, (u64)(((u128)1 << 32) % qt), qt);
      e[2] = (double)dm[2 * m];
    }
  t.hat_f = (double*)c->table_upload(hf.data(), hf.size() * 8);
  return t;
}

// Digit tables of the MFMA form of ModDown's lift (sources of at most 63
// bits: nine 7-bit digits each; targets of at most 46 bits: seven digits).
static void fbc_digits(HeCtxImpl* c, FbcTable& t) {
  if (t.ns < 1 || t.ns > 4) return;
  const int kb = 9 * t.ns + 1;
  t.kw = 2 * ((kb + 15) / 16);
  std::vector<u64> cd((size_t)c->nmods * 8 * t.kw, 0);
  for (int m = 0; m < c->nmods; m++) {
    const u64 qt = c->mods[m];
    if (qt >> 46) continue;  // only targets of the FP64 path use the table
    u64 d = 1;
    for (int a = 0; a < t.ns; a++) d = hmul(d, c->mods[t.src[a]] % qt, qt);
    for (int k = 0; k < kb; k++) {
      u64 cst;
      if (k == 9 * t.ns) {
        cst = d == 0 ? 0 : qt - d;
      } else {
        const int a = k / 9, i = k % 9;
        u64 h = 1;
        for (int b = 0; b < t.ns; b++)
          if (b != a) h = hmul(h, c->mods[t.src[b]] % qt, qt);
        cst = hmul(h, (u64)(((u128)1 << (7 * i)) % qt), qt);
      }
      for (int j = 0; j < 7; j++) {
        const u64 dig = (cst >> (7 * j)) & 127;
        cd[((size_t)m * 8 + j) * t.kw + k / 8] |= dig << (8 * (k % 8));
      }
    }
  }
  t.cdig = c->table_upload(cd.data(), cd.size() * 8);
}

void HeCtxImpl::init(const he_params* p, const he_device* dev, u64 seed_) {
  if (!p || p->log_n < 10 || p->log_n > 16) fail(HE_EINVAL, "log_n must be in [10, 16]");
  if (p->n_q < 1 || p->n_q > 48 || p->n_p < 1 || p->n_p > 4) fail(HE_EINVAL, "1..48 Q primes and 1..4 P primes");
  logN = (int)p->log_n;
  N = 1ull << logN;
  L = (int)p->n_q - 1;
  alpha = (int)p->n_p;
  beta = (L + alpha) / alpha;
  fused_conv = logN >= 12 && logN <= 16;
  if (beta > 16) fail(HE_EINVAL, "at most 16 decomposition digits");
  nmods = L + 1 + alpha;
  std::vector<int> bits;
  for (u32 k = 0; k < p->n_q; k++) bits.push_back((int)p->q_bits[k]);
  for (u32 k = 0; k < p->n_p; k++) bits.push_back((int)p->p_bits[k]);
  for (int b : bits)
    if (b < 30 || b > 61) fail(HE_EINVAL, "prime sizes must be 30..61 bits");
  choose_primes(logN, bits, mods);
  delta = std::pow(2.0, p->log2_scale);
  sigma = p->sigma;
  seed = seed_;

  if (dev) {
    pool.user_alloc = dev->alloc;
    pool.user_release = dev->release;
    pool.user = dev->user;
    stream = (hipStream_t)dev->hip_stream;
  }
  if (!stream) {
    hip_check(hipStreamCreateWithFlags(&stream, hipStreamNonBlocking), "stream");
    own_stream = true;
  }
  pool.stream = stream;
  hip_check(hipStreamCreateWithFlags(&fork.aux, hipStreamNonBlocking), "stream");
  hip_check(hipEventCreateWithFlags(&fork.fork, hipEventDisableTiming), "event");
  hip_check(hipEventCreateWithFlags(&fork.join, hipEventDisableTiming), "event");
  hip_check(hipEventCreate(&ev0), "event");
  hip_check(hipEventCreate(&ev1), "event");

  // per-modulus constants and NTT twiddles (Shoup pairs)
  mc.resize(nmods);
  std::vector<u64> psi((size_t)nmods * N), psi_sh((size_t)nmods * N), ipsi((size_t)nmods * N),
      ipsi_sh((size_t)nmods * N);
  for (int m = 0; m < nmods; m++) {
    u64 q = mods[m];
    ModConst& k = mc[m];
    k.q = q;
    k.bits = 64 - __builtin_clzll(q);
    k.mu = (u64)(((u128)1 << (2 * k.bits)) / q);
    k.ninv = hinv(N % q, q);
    k.ninv_sh = shoup_pre(k.ninv, q);
    k.r64 = (u64)(((u128)1 << 64) % q);
    k.r64_sh = shoup_pre(k.r64, q);
    k.r96 = (u64)(((u128)k.r64 << 32) % q);
    k.qf = (double)q;
    k.qinvf = 1.0 / k.qf;
    u64 w = root_2n(q, logN), wi = hinv(w, q);
    for (u64 i = 0; i < N; i++) {
      u32 e = brv_host((u32)i, logN);
      u64 a = hpow(w, e, q), b = hpow(wi, e, q);
      psi[(size_t)m * N + i] = a;
      psi_sh[(size_t)m * N + i] = shoup_pre(a, q);
      ipsi[(size_t)m * N + i] = b;
      ipsi_sh[(size_t)m * N + i] = shoup_pre(b, q);
    }
  }
  T.logN = logN;
  T.N = N;
  T.nmods = nmods;
  T.mc = (ModConst*)table_upload(mc.data(), sizeof(ModConst) * nmods);
  for (int m = 0; m < nmods; m++) T.bits[m] = (int)mc[m].bits;
  T.psi = table_upload(psi.data(), psi.size() * 8);
  T.psi_sh = table_upload(psi_sh.data(), psi_sh.size() * 8);
  T.ipsi = table_upload(ipsi.data(), ipsi.size() * 8);
  T.ipsi_sh = table_upload(ipsi_sh.data(), ipsi_sh.size() * 8);
  {
    std::vector<double> pf(psi.size()), ipf(ipsi.size());
    for (size_t i = 0; i < psi.size(); i++) {
      pf[i] = (double)psi[i];
      ipf[i] = (double)ipsi[i];
    }
    T.psi_f = (double*)table_upload(pf.data(), pf.size() * 8);
    T.ipsi_f = (double*)table_upload(ipf.data(), ipf.size() * 8);
  }

  // canonical embedding tables
  std::vector<double> tw(N / 2 * 4), zt(N * 4);
  he_host_dd_tables(logN, tw.data(), zt.data());
  T.fft_tw = (double*)table_upload(tw.data(), tw.size() * 8);
  T.zeta = (double*)table_upload(zt.data(), zt.size() * 8);
  std::vector<u32> rg(N / 2);
  u64 g = 1;
  for (u64 j = 0; j < N / 2; j++) {
    rg[j] = (u32)g;
    g = (g * 5) % (2 * N);
  }
  T.rotgroup = (u32*)table_upload(rg.data(), rg.size() * 4);

  // Gaussian inversion table for chi_e: cumulative discrete Gaussian, |e| <= 19
  {
    double rho[39], z = 0.0;
    for (int x = -19; x <= 19; x++) rho[x + 19] = std::exp(-((double)x * (double)x) / (2.0 * sigma * sigma));
    for (int k = 0; k < 39; k++) z += rho[k];
    u64 cdt[38];
    double cum = 0.0;
    for (int k = 0; k < 38; k++) {
      cum += rho[k];
      cdt[k] = (u64)(cum / z * 18446744073709551616.0);
    }
    T.cdt = table_upload(cdt, sizeof cdt);
  }

  // ModUp tables per (level, digit); ModDown table P -> Q
  up.resize(L + 1);
  for (int l = 0; l <= L; l++) {
    for (int j = 0; j < beta_at(l); j++) {
      std::vector<int> src;
      for (int k = j * alpha; k < (j + 1) * alpha && k <= l; k++) src.push_back(k);
      up[l].push_back(make_fbc(this, src));
    }
  }
  {
    std::vector<int> src;
    for (int k = 0; k < alpha; k++) src.push_back(L + 1 + k);
    down = make_fbc(this, src);
    fbc_digits(this, down);
  }
  // ModDown + Rescale as one rounding: sources q_l and P (at most 4 limbs)
  if (alpha <= 3) {
    down_rs.resize(L + 1);
    for (int l = 1; l <= L; l++) {
      std::vector<int> src{l};
      for (int k = 0; k < alpha; k++) src.push_back(L + 1 + k);
      down_rs[l] = make_fbc(this, src);
      fbc_digits(this, down_rs[l]);
    }
  }
  // P mod q, P^{-1} mod q (Shoup pairs) and q_l^{-1} mod q_k
  std::vector<u64> pm(2 * nmods), pi(2 * nmods), ql((size_t)nmods * nmods * 2);
  for (int m = 0; m < nmods; m++) {
    u64 q = mods[m], P = 1;
    for (int k = 0; k < alpha; k++) P = hmul(P, mods[L + 1 + k] % q, q);
    pm[2 * m] = P;
    pm[2 * m + 1] = shoup_pre(P, q);
    u64 Pi = m <= L ? hinv(P, q) : 0;
    pi[2 * m] = Pi;
    pi[2 * m + 1] = shoup_pre(Pi, q);
  }
  for (int l = 0; l < nmods; l++)
    for (int k = 0; k < nmods; k++) {
      u64 v = k == l ? 0 : hinv(mods[l] % mods[k], mods[k]);
      ql[((size_t)l * nmods + k) * 2] = v;
      ql[((size_t)l * nmods + k) * 2 + 1] = shoup_pre(v, mods[k]);
    }
  pmod = DevBuf(&pool, pm.size());
  hip_check(hipMemcpy(pmod.p, pm.data(), pm.size() * 8, hipMemcpyHostToDevice), "pmod");
  pinv = DevBuf(&pool, pi.size());
  hip_check(hipMemcpy(pinv.p, pi.data(), pi.size() * 8, hipMemcpyHostToDevice), "pinv");
  qlinv = DevBuf(&pool, ql.size());
  hip_check(hipMemcpy(qlinv.p, ql.data(), ql.size() * 8, hipMemcpyHostToDevice), "qlinv");
  {
    std::vector<u64> pq((size_t)(L + 1) * nmods * 2, 0);
    for (int l = 1; l <= L; l++)
      for (int k = 0; k < l; k++) {
        const u64 q = mods[k];
        const u64 v = hinv(hmul(pm[2 * k], mods[l] % q, q), q);
        pq[((size_t)l * nmods + k) * 2] = v;
        pq[((size_t)l * nmods + k) * 2 + 1] = shoup_pre(v, q);
      }
    pqlinv = DevBuf(&pool, pq.size());
    hip_check(hipMemcpy(pqlinv.p, pq.data(), pq.size() * 8, hipMemcpyHostToDevice), "pqlinv");
  }
  {
    // Decompose's inverse transform ends with N^-1 times limb t's hat inverse
    // in its digit (one constant a limb, Shoup pairs)
    std::vector<u64> us((size_t)(L + 1) * nmods * 2, 0);
    for (int l = 0; l <= L; l++)
      for (int t = 0; t <= l; t++) {
        const u64 q = mods[t];
        const u64 v = hmul(hinv(N % q, q), up[l][t / alpha].hatinv[t % alpha], q);
        us[((size_t)l * nmods + t) * 2] = v;
        us[((size_t)l * nmods + t) * 2 + 1] = shoup_pre(v, q);
      }
    up_scale = DevBuf(&pool, us.size());
    hip_check(hipMemcpy(up_scale.p, us.data(), us.size() * 8, hipMemcpyHostToDevice), "up_scale");
  }
  hip_check(hipDeviceSynchronize(), "init");
}

// ---------------------------------------------------------------------------
// basic containers
// ---------------------------------------------------------------------------
HeCt HeCtxImpl::ct_new(int level, bool qp, double scale, int B) {
  HeCt c;
  c.N = N;
  c.level = level;
  c.qp = qp;
  c.nlimbs = level + 1 + (qp ? alpha : 0);
  c.B = B;
  c.scale = scale;
  c.d = DevBuf(&pool, (size_t)2 * B * c.nlimbs * N);
  return c;
}
HeCt HeCtxImpl::ct_copy(const HeCt& x) {
  HeCt c = ct_new(x.level, x.qp, x.scale, x.B);
  hip_check(copy_async("copy_ct", c.d.p, x.d.p, c.d.words * 8, stream), "copy");
  c.packed = x.packed;
  return c;
}
void HeCtxImpl::copy_limbs(u64* dst, const u64* src, size_t nlimbs, const char* family) {
  hip_check(copy_async(family, dst, src, nlimbs * N * 8, stream), "copy");
}

// ---------------------------------------------------------------------------
// encoding
// ---------------------------------------------------------------------------
DevBuf HeCtxImpl::encode_batch(const double* z_host, int nz, int batch, double dlt) {
  if (nz <= 0 || (N / 2) % (u64)nz) fail(HE_EINVAL, "message length must divide N/2");
  DevBuf zd;
  zd = DevBuf(&pool, (size_t)nz * batch);
  hip_check(hipMemcpyAsync(zd.p, z_host, (size_t)nz * batch * 8, hipMemcpyHostToDevice, stream), "z upload");
  DevBuf out(&pool, (size_t)batch * N);
  DevBuf scratch(&pool, encode_scratch_bytes(T, batch) / 8);
  launch_encode(T, (i64*)out.p, (const double*)zd.p, nz, batch, dlt, scratch.p, stream);
  // the host buffer may be reused by the caller once the copy is done
  hip_check(hipStreamSynchronize(stream), "encode");
  return out;
}

// integer coefficients -> evaluation-domain limbs for the map's moduli
void HeCtxImpl::int_to_ntt(u64* out, const i64* m, const LimbMap& map) {
  launch_int_to_limbs(T, out, m, map.n, map, stream);
  launch_ntt(T, out, map.n, map, false, stream);
}

// ---------------------------------------------------------------------------
// key generation (Appendix A)
// ---------------------------------------------------------------------------
void HeCtxImpl::keygen_secret() {
  if (have_sk) return;
  DevBuf si(&pool, N);
  launch_sample_ternary(T, (i64*)si.p, seed, TAG_SK, 0, 0, 0, stream);
  s_ntt = DevBuf(&pool, (size_t)nmods * N);
  LimbMap all;
  all.n = nmods;
  for (int m = 0; m < nmods; m++) all.idx[m] = (short)m;
  int_to_ntt(s_ntt.p, (const i64*)si.p, all);
  // public key (-a s + e, a) over Q_L
  pk = DevBuf(&pool, (size_t)2 * (L + 1) * N);
  u64* a = pk.p + (size_t)(L + 1) * N;
  LimbMap qm = qmap(L + 1);
  launch_sample_uniform(T, a, L + 1, qm, seed, TAG_PK_A, 0, 0, stream);
  DevBuf e(&pool, N), en(&pool, (size_t)(L + 1) * N);
  launch_sample_gauss(T, (i64*)e.p, seed, TAG_PK_E, 0, 0, 0, stream);
  int_to_ntt(en.p, (const i64*)e.p, qm);
  launch_swk_b(T, pk.p, a, en.p, s_ntt.p, nullptr, pmod.p, L + 1, 0, alpha, L, stream);
  have_sk = true;
}

// switching key from s' (evaluation domain over all moduli) to s
void HeCtxImpl::swk_gen(const u64* sp, u64 kid, DevBuf& out) {
  out = DevBuf(&pool, (size_t)beta * 2 * nmods * N);
  LimbMap all;
  all.n = nmods;
  for (int m = 0; m < nmods; m++) all.idx[m] = (short)m;
  DevBuf e(&pool, N), en(&pool, (size_t)nmods * N);
  for (int j = 0; j < beta; j++) {
    u64* bj = out.p + ((size_t)j * 2 + 0) * nmods * N;
    u64* aj = out.p + ((size_t)j * 2 + 1) * nmods * N;
    launch_sample_uniform(T, aj, nmods, all, seed, TAG_SWK_A, (u64)j, kid, stream);
    launch_sample_gauss(T, (i64*)e.p, seed, TAG_SWK_E, 0, (u64)j, kid, stream);
    int_to_ntt(en.p, (const i64*)e.p, all);
    launch_swk_b(T, bj, aj, en.p, s_ntt.p, sp, pmod.p, nmods, j, alpha, L, stream);
  }
  launch_key_f64(T, out.p, beta * 2, nmods, stream);
}

void HeCtxImpl::keygen_relin() {
  if (keys.count(0)) return;
  LimbMap all;
  all.n = nmods;
  for (int m = 0; m < nmods; m++) all.idx[m] = (short)m;
  DevBuf s2(&pool, (size_t)nmods * N);
  launch_mul(T, s2.p, s_ntt.p, s_ntt.p, nmods, all, stream);
  swk_gen(s2.p, 0, keys[0]);
}

void HeCtxImpl::keygen_rot(long step) {
  u64 g = galois(step);
  if (g == 1 || keys.count(g)) return;
  DevBuf sg(&pool, (size_t)nmods * N);
  launch_automorph(T, sg.p, s_ntt.p, nmods, g, stream);
  swk_gen(sg.p, g, keys[g]);
}

const DevBuf& HeCtxImpl::key(u64 g) {
  auto it = keys.find(g);
  if (it == keys.end()) fail(HE_EKEY, "missing switching key for Galois element " + std::to_string(g));
  return it->second;
}

// ---------------------------------------------------------------------------
// encryption / decryption (Appendix A: Enc, Dec)
// ---------------------------------------------------------------------------
HeCt HeCtxImpl::encrypt_int(const i64* m_dev, int level, double scale, u64 nonce) {
  if (!have_sk) fail(HE_EKEY, "keys not generated");
  if (level < 0 || level > L) fail(HE_ELEVEL, "level out of range");
  int nl = level + 1;
  LimbMap qm = qmap(nl);
  DevBuf v(&pool, N), e0(&pool, N), e1(&pool, N);
  launch_sample_ternary(T, (i64*)v.p, seed, TAG_ENC_V, 0, nonce, 0, stream);
  launch_sample_gauss(T, (i64*)e0.p, seed, TAG_ENC_E0, 0, nonce, 0, stream);
  launch_sample_gauss(T, (i64*)e1.p, seed, TAG_ENC_E1, 0, nonce, 0, stream);
  launch_add_int((i64*)e0.p, (const i64*)e0.p, m_dev, N, stream);
  DevBuf vn(&pool, (size_t)nl * N);
  int_to_ntt(vn.p, (const i64*)v.p, qm);
  HeCt c = ct_new(level, false, scale);
  int_to_ntt(c.poly(0), (const i64*)e0.p, qm);
  int_to_ntt(c.poly(1), (const i64*)e1.p, qm);
  // c0 += v pk0 ; c1 += v pk1  (pk rows restricted to the first nl limbs)
  launch_mul_acc(T, c.poly(0), vn.p, pk.p, nl, nl, qm, stream);
  launch_mul_acc(T, c.poly(1), vn.p, pk.p + (size_t)(L + 1) * N, nl, nl, qm, stream);
  return c;
}

HeCt HeCtxImpl::encrypt(const double* z, int nz, int level, u64 nonce) {
  DevBuf m = encode_batch(z, nz, 1, delta);
  return encrypt_int((const i64*)m.p, level, delta, nonce);
}

std::vector<double> HeCtxImpl::decrypt(const HeCt& c) {
  if (!have_sk) fail(HE_EKEY, "keys not generated");
  if (c.qp) fail(HE_EINVAL, "cannot decrypt an R_QP element");
  if (c.B != 1) fail(HE_EINVAL, "decrypt takes a single ciphertext, not a batch");
  DevBuf t(&pool, N);
  LimbMap m0 = one(0);
  launch_mul(T, t.p, c.limb(1, 0), s_ntt.p, 1, m0, stream);
  launch_add(T, t.p, t.p, c.limb(0, 0), 1, m0, stream);
  launch_ntt(T, t.p, 1, m0, true, stream);
  DevBuf mi(&pool, N);
  launch_centre_to_int(T, (i64*)mi.p, t.p, 0, stream);
  double inv = 1.0 / c.scale;
  DevBuf invd(&pool, 1);
  hip_check(hipMemcpyAsync(invd.p, &inv, 8, hipMemcpyHostToDevice, stream), "scale");
  DevBuf out(&pool, N / 2);
  DevBuf scratch(&pool, encode_scratch_bytes(T, 1) / 8);
  launch_decode(T, (double*)out.p, (const i64*)mi.p, 1, (const double*)invd.p, scratch.p, stream);
  std::vector<double> h(N / 2);
  hip_check(hipMemcpyAsync(h.data(), out.p, (N / 2) * 8, hipMemcpyDeviceToHost, stream), "download");
  hip_check(hipStreamSynchronize(stream), "decrypt");
  return h;
}

// ---------------------------------------------------------------------------
// Add / Sub / PMult / Mult / Rescale / level drop (B members at once)
// ---------------------------------------------------------------------------
static void need_same(const HeCt& a, const HeCt& b) {
  if (a.level != b.level || a.qp != b.qp) fail(HE_ELEVEL, "operands at different levels");
  if (a.B != b.B) fail(HE_EINVAL, "operands with different batch sizes");
}
HeCt HeCtxImpl::add(const HeCt& a, const HeCt& b, bool sub) {
  need_same(a, b);
  if (a.scale != b.scale) fail(HE_ESCALE, "operands with different scales");
  HeCt c = ct_new(a.level, a.qp, a.scale, a.B);
  LimbMap m = a.qp ? qpmap(a.level) : qmap(a.level + 1);
  const int nl = (int)a.polys() * a.nlimbs;
  if (sub) launch_sub(T, c.d.p, a.d.p, b.d.p, nl, m, stream);
  else launch_add(T, c.d.p, a.d.p, b.d.p, nl, m, stream);
  return c;
}
void HeCtxImpl::add_into(HeCt& acc, const HeCt& b) {
  need_same(acc, b);
  if (acc.packed || b.packed) fail(HE_EINVAL, "packed limbs are for the tensor sums alone");
  LimbMap m = acc.qp ? qpmap(acc.level) : qmap(acc.level + 1);
  launch_add(T, acc.d.p, acc.d.p, b.d.p, (int)acc.polys() * acc.nlimbs, m, stream);
}

// the first `count` limbs of every poly of x into dst [polys][count][N]
void HeCtxImpl::gather_limbs(u64* dst, const HeCt& x, int first, int count) {
  hip_check(copy2d_async("copy_gather", dst, (size_t)count * N * 8, x.d.p + (size_t)first * N,
                         (size_t)x.nlimbs * N * 8, (size_t)count * N * 8, x.polys(), stream),
            "gather");
}

HeCt HeCtxImpl::drop(const HeCt& a, int level) {
  if (a.qp || level > a.level || level < 0) fail(HE_ELEVEL, "bad level drop");
  HeCt c = ct_new(level, false, a.scale, a.B);
  gather_limbs(c.d.p, a, 0, level + 1);
  c.packed = a.packed;  // whole limb slots copied
  return c;
}

// Rescale by q_l; out_level < l - 1 also drops the limbs above it (only the
// kept limbs are computed: the same residues as Rescale followed by a drop)
HeCt HeCtxImpl::rescale(const HeCt& a, int out_level) {
  if (a.qp) fail(HE_EINVAL, "rescale of an R_QP element");
  if (a.packed) fail(HE_EINVAL, "packed limbs are for the tensor sums alone");
  int l = a.level;
  if (l < 1) fail(HE_ELEVEL, "no level left to rescale");
  if (out_level < 0) out_level = l - 1;
  if (out_level > l - 1) fail(HE_ELEVEL, "rescale cannot raise the level");
  const int np = (int)a.polys(), nout = out_level + 1;
  DevBuf top(&pool, (size_t)np * N);
  gather_limbs(top.p, a, l, 1);
  launch_ntt(T, top.p, np, one(l), true, stream);
  DevBuf t(&pool, (size_t)np * nout * N);
  HeCt c = ct_new(out_level, false, a.scale / (double)mods[l], a.B);
  const u64* ql_inv = qlinv.p + (size_t)l * nmods * 2;
  if (fused_conv) {
    if (!launch_rescale_fused(T, t.p, top.p, l, nout, np, a.d.p, l + 1, ql_inv, c.d.p, stream))
      fail(HE_EINVAL, "fused Rescale unavailable for this ring size");
    return c;
  }
  launch_rescale_lift(T, t.p, top.p, l, nout, np, stream);
  launch_ntt_fwd_sub(T, t.p, nout, np, qmap(nout), a.d.p, l + 1, ql_inv, c.d.p, stream);
  return c;
}

// ---------------------------------------------------------------------------
// key switching (section 3.3.1; Appendix A KeySwitch)
// ---------------------------------------------------------------------------
// Decompose B polynomials d [B][l+1][N]: digits u64[B][beta_l][l+1+alpha][N], evaluation domain
// Decompose: the digits [B][beta_l][nqp][N] in the evaluation domain, limbs
// of moduli below 2^46 as centred doubles (the key inner products' operand
// form), the others as residues in [0, q)
DevBuf HeCtxImpl::decompose(const u64* d, int level, int B) {
  int nq = nq_of(level), nqp = nqp_of(level), bl = beta_at(level);
  DevBuf coef(&pool, (size_t)B * nq * N);
  if (!fused_conv) {
    copy_limbs(coef.p, d, (size_t)B * nq, "copy_decompose");
    launch_ntt(T, coef.p, B * nq, qmap(nq), true, stream);
  }
  DevBuf dig(&pool, (size_t)B * bl * nqp * N);
  LimbMap m;
  m.n = bl * nqp;
  if (m.n > 960) fail(HE_EINVAL, "too many digit limbs");
  for (int j = 0; j < bl; j++)
    for (int pos = 0; pos < nqp; pos++) {
      bool own = pos < nq && pos / alpha == j;
      m.idx[j * nqp + pos] = own ? (short)-1 : (short)qp_mod(level, pos);
    }
  if (fused_conv) {
    // sources times their hat inverses (the inverse transform's last scaling,
    // read from d directly), then conversion + NTT in one pass pair
    const std::vector<FbcTable>& tabs = up[level];
    if (!launch_intt_scaled(T, coef.p, d, B * nq, qmap(nq), up_scale.p + (size_t)level * nmods * 2, stream)) {
      std::vector<u64> hinv((size_t)2 * nq);
      for (int t = 0; t < nq; t++) {
        hinv[2 * t] = tabs[t / alpha].hatinv[t % alpha];
        hinv[2 * t + 1] = tabs[t / alpha].hatinv_sh[t % alpha];
      }
      copy_limbs(coef.p, d, (size_t)B * nq, "copy_decompose");
      launch_ntt(T, coef.p, B * nq, qmap(nq), true, stream);
      launch_mul_const(T, coef.p, coef.p, B * nq, hinv.data(), qmap(nq), stream);
    }
    if (launch_modup_ntt(T, dig.p, coef.p, d, level, L, alpha, bl, tabs.data(), B, m, stream)) {
      n_decompose += B;
      return dig;
    }
    fail(HE_EINVAL, "fused decomposition unavailable for this ring size");
  }
  launch_modup(T, dig.p, coef.p, d, level, L, alpha, bl, up[level].data(), B, stream);
  launch_ntt(T, dig.p, B * m.n, m, false, stream);
  LimbMap all;
  all.n = bl * nqp;
  for (int j = 0; j < bl; j++)
    for (int pos = 0; pos < nqp; pos++) all.idx[j * nqp + pos] = (short)qp_mod(level, pos);
  launch_digits_f64(T, dig.p, B * all.n, all, stream);
  n_decompose += B;
  return dig;
}

// hoisted rotation left in R_{Q_l P}; g = 1 gives the P-lift
HeCt HeCtxImpl::hoisted(const HeCt& x, const u64* digits, u64 g) {
  HeCt h = ct_new(x.level, true, x.scale, x.B);
  if (g == 1) {
    launch_plift(T, h.d.p, x.d.p, pmod.p, x.level, alpha, (int)x.polys(), stream);
    return h;
  }
  const DevBuf& k = key(g);
  launch_multsum(T, h.d.p, digits, k.p, x.poly(0), pmod.p, x.level, L, alpha, beta_at(x.level), g, x.B, stream);
  n_multsum += x.B;
  return h;
}

// several hoisted rotations of one decomposition (one launch for all of them)
std::vector<HeCt> HeCtxImpl::hoisted_multi(const HeCt& x, const u64* digits, const std::vector<u64>& gs) {
  std::vector<HeCt> out(gs.size());
  std::vector<u64*> outs;
  std::vector<const u64*> ks;
  std::vector<u64> g2;
  for (size_t r = 0; r < gs.size(); r++) {
    out[r] = ct_new(x.level, true, x.scale, x.B);
    if (gs[r] == 1) {
      launch_plift(T, out[r].d.p, x.d.p, pmod.p, x.level, alpha, (int)x.polys(), stream);
      continue;
    }
    outs.push_back(out[r].d.p);
    ks.push_back(key(gs[r]).p);
    g2.push_back(gs[r]);
  }
  if (!outs.empty())
    launch_multsum_rot(T, outs.data(), ks.data(), g2.data(), (int)outs.size(), digits, x.poly(0), pmod.p, x.level,
                       L, alpha, beta_at(x.level), x.B, stream, nullptr, false, &fork);
  n_multsum += (long)x.B * (long)outs.size();
  return out;
}

// hoisted rotations of one decomposition, each multiplied by its mask (a
// plaintext in R_{Q_l P}) and written to (or, accumulate, added onto) outs[r]
void HeCtxImpl::hoisted_masked(const HeCt& x, const u64* digits, const std::vector<u64>& gs,
                               const std::vector<u64*>& outs, const std::vector<const u64*>& masks, bool accumulate) {
  if (gs.empty()) return;
  std::vector<const u64*> ks;
  for (u64 g : gs) {
    if (g == 1) fail(HE_EINVAL, "masked hoisted rotation by the identity");
    ks.push_back(key(g).p);
  }
  launch_multsum_rot(T, outs.data(), ks.data(), gs.data(), (int)gs.size(), digits, x.poly(0), pmod.p, x.level, L,
                     alpha, beta_at(x.level), x.B, stream, masks.data(), accumulate, &fork);
  n_multsum += (long)x.B * (long)gs.size();
}

// outs[r] = m1[r] (rotation gs[r] of x) + m2[r] (rotation gs[r] of y): one
// multi-rotation launch over both decompositions; false where that does not
// apply (nothing launched)
bool HeCtxImpl::hoisted_masked_pair(const HeCt& x, const u64* dx, const std::vector<const u64*>& m1, const HeCt& y,
                                    const u64* dy, const std::vector<const u64*>& m2, const std::vector<u64>& gs,
                                    const std::vector<u64*>& outs) {
  if (gs.empty()) return true;
  if (x.level != y.level || x.B != y.B) fail(HE_EINVAL, "paired bases of unlike elements");
  std::vector<const u64*> ks;
  for (u64 g : gs) {
    if (g == 1) fail(HE_EINVAL, "masked hoisted rotation by the identity");
    ks.push_back(key(g).p);
  }
  if (!launch_multsum_rot_pair(T, outs.data(), ks.data(), gs.data(), (int)gs.size(), dx, x.poly(0), m1.data(), dy,
                               y.poly(0), m2.data(), pmod.p, x.level, L, alpha, beta_at(x.level), x.B, stream))
    return false;
  n_multsum += 2L * x.B * (long)gs.size();
  return true;
}

// ModDown: R_{Q_l P}^2 -> R_{Q_l}^2, (x - [x]_P) P^{-1} with [x]_P the exact
// centred residue; out_level < l keeps (and computes) only the limbs up to it
HeCt HeCtxImpl::moddown(const HeCt& x, int out_level, bool consume, bool src_ready, const u64* rec, bool pack) {
  if (!x.qp) fail(HE_EINVAL, "moddown of an R_Q element");
  if (out_level < 0) out_level = x.level;
  if (out_level > x.level) fail(HE_ELEVEL, "moddown cannot raise the level");
  HeCt c = ct_new(out_level, false, x.scale, x.B);
  c.packed = moddown_to(x, out_level, c.d.p, consume, src_ready, rec, pack);
  return c;
}
// the same into out [2][B][out_level + 1][N].  consume: x's special-prime
// limbs are brought to the coefficient domain in place (x is left with them
// so) instead of in a gathered copy; src_ready: that was done already
// (moddown_sources over a set of elements), and rec, when given, holds their
// digit records
bool HeCtxImpl::moddown_to(const HeCt& x, int out_level, u64* out, bool consume, bool src_ready, const u64* rec,
                           bool pack) {
  int nq = nq_of(out_level), nqp = nqp_of(x.level);
  const int np = (int)x.polys();
  DevBuf y(&pool, (size_t)np * nq * N);
  LimbMap pm;
  pm.n = alpha;
  for (int k = 0; k < alpha; k++) pm.idx[k] = (short)(L + 1 + k);
  if (fused_conv && consume) {
    pm.slot_per = (short)alpha;
    pm.slot_stride = (short)x.nlimbs;
    pm.slot_off = (short)nq_of(x.level);
    if (!src_ready) launch_ntt(T, x.d.p, np * alpha, pm, true, stream);
    DevBuf V;
    if (!rec) V = DevBuf(&pool, (size_t)np * (down.ns + 1) * N);
    if (!launch_moddown_fused(T, x.d.p, nq, np, down, x.d.p, nqp, pinv.p, out, y.p, rec ? (u64*)rec : V.p, stream,
                              x.nlimbs, nq_of(x.level), rec != nullptr, pack))
      fail(HE_EINVAL, "fused ModDown unavailable for this ring size");
    n_moddown += x.B;
    return pack;
  }
  DevBuf pc(&pool, (size_t)np * alpha * N);
  gather_limbs(pc.p, x, nq_of(x.level), alpha);
  launch_ntt(T, pc.p, np * alpha, pm, true, stream);
  if (fused_conv) {
    DevBuf V(&pool, (size_t)np * (down.ns + 1) * N);
    if (!launch_moddown_fused(T, pc.p, nq, np, down, x.d.p, nqp, pinv.p, out, y.p, V.p, stream))
      fail(HE_EINVAL, "fused ModDown unavailable for this ring size");
  } else {
    launch_fbc_to_q(T, y.p, pc.p, nq, np, down, stream);
    launch_ntt_fwd_sub(T, y.p, nq, np, qmap(nq), x.d.p, nqp, pinv.p, out, stream);
  }
  n_moddown += x.B;
  return false;
}

// ModDown and the Rescale after it as one rounding: x in R_{Q_l P} ->
// round(x / (P q_l)) in R_{Q_{l-1}} (or a lower out_level: only the kept
// limbs are computed): the exact centred lift of x mod P q_l from the limbs
// q_l, p_1..p_alpha, then (x - lift) (P q_l)^-1 on the limbs below q_l.
HeCt HeCtxImpl::moddown_rescale(const HeCt& x, int out_level, bool consume, bool src_ready, const u64* rec,
                                 bool pack) {
  if (!x.qp) fail(HE_EINVAL, "moddown of an R_Q element");
  const int l = x.level;
  if (l < 1) fail(HE_ELEVEL, "no level left to rescale");
  if (down_rs.empty()) fail(HE_EINVAL, "one rounding for ModDown and Rescale needs at most 3 special primes");
  if (out_level < 0) out_level = l - 1;
  if (out_level > l - 1) fail(HE_ELEVEL, "rescale cannot raise the level");
  const int nqx = nq_of(l), nqp = nqp_of(l), nout = out_level + 1, ns = alpha + 1;
  const int np = (int)x.polys();
  const FbcTable& tab = down_rs[l];
  LimbMap sm;
  sm.n = ns;
  sm.idx[0] = (short)l;
  for (int k = 0; k < alpha; k++) sm.idx[1 + k] = (short)(L + 1 + k);
  const u64* cp = pqlinv.p + (size_t)l * nmods * 2;
  if (fused_conv && consume) {
    // q_l and the special primes are the consecutive slots l .. l + alpha of
    // each poly: transformed in place, read from there
    sm.slot_per = (short)ns;
    sm.slot_stride = (short)x.nlimbs;
    sm.slot_off = (short)l;
    if (!src_ready) launch_ntt(T, x.d.p, np * ns, sm, true, stream);
    DevBuf y(&pool, (size_t)np * nout * N);
    HeCt c = ct_new(out_level, false, x.scale / (double)mods[l], x.B);
    DevBuf V;
    if (!rec) V = DevBuf(&pool, (size_t)np * (ns + 1) * N);
    if (!launch_moddown_fused(T, x.d.p, nout, np, tab, x.d.p, nqp, cp, c.d.p, y.p, rec ? (u64*)rec : V.p, stream,
                              x.nlimbs, l, rec != nullptr, pack))
      fail(HE_EINVAL, "fused ModDown unavailable for this ring size");
    c.packed = pack;
    n_moddown += x.B;
    return c;
  }
  // sources [np][q_l, p_1..p_alpha] in the coefficient domain
  DevBuf pc(&pool, (size_t)np * ns * N);
  hip_check(copy2d_async("copy_gather", pc.p, (size_t)ns * N * 8, x.d.p + (size_t)l * N, (size_t)x.nlimbs * N * 8,
                         (size_t)N * 8, np, stream),
            "gather");
  hip_check(copy2d_async("copy_gather", pc.p + N, (size_t)ns * N * 8, x.d.p + (size_t)nqx * N,
                         (size_t)x.nlimbs * N * 8, (size_t)alpha * N * 8, np, stream),
            "gather");
  launch_ntt(T, pc.p, np * ns, sm, true, stream);
  DevBuf y(&pool, (size_t)np * nout * N);
  HeCt c = ct_new(out_level, false, x.scale / (double)mods[l], x.B);
  if (fused_conv) {
    DevBuf V(&pool, (size_t)np * (ns + 1) * N);
    if (!launch_moddown_fused(T, pc.p, nout, np, tab, x.d.p, nqp, cp, c.d.p, y.p, V.p, stream))
      fail(HE_EINVAL, "fused ModDown unavailable for this ring size");
  } else {
    launch_fbc_to_q(T, y.p, pc.p, nout, np, tab, stream);
    launch_ntt_fwd_sub(T, y.p, nout, np, qmap(nout), x.d.p, nqp, cp, c.d.p, stream);
  }
  n_moddown += x.B;
  return c;
}

// The ModDown sources of a set of R_{Q_l P} elements of one level and batch,
// brought to the coefficient domain in place by one launch per 64 elements:
// the special-prime limbs, and q_l too when the ModDown is fused with the
// Rescale.  The elements are then ModDown'ed with consume and src_ready.
// Where the ModDown takes digit records (the int8 lift into every target
// limb up to the elements' level), the transform's last pass writes the
// records instead of the limbs, and they are returned for the ModDowns
// (element e's at rec + e * rec_stride).
DevBuf HeCtxImpl::moddown_sources(const std::vector<HeCt*>& xs, bool with_rescale, size_t* rec_stride) {
  if (xs.empty() || !fused_conv) return DevBuf();
  const HeCt& x0 = *xs[0];
  std::vector<u64*> bases;
  for (HeCt* x : xs) {
    if (!x->qp || x->level != x0.level || x->B != x0.B) fail(HE_EINVAL, "moddown sources of unlike elements");
    bases.push_back(x->d.p);
  }
  const int l = x0.level, np = (int)x0.polys();
  LimbMap m;
  const FbcTable* tab;
  int per, off, nq;
  if (with_rescale) {
    m.n = per = alpha + 1;
    m.idx[0] = (short)l;
    for (int k = 0; k < alpha; k++) m.idx[1 + k] = (short)(L + 1 + k);
    tab = &down_rs[l];
    off = l;
    nq = l;
  } else {
    m.n = per = alpha;
    for (int k = 0; k < alpha; k++) m.idx[k] = (short)(L + 1 + k);
    tab = &down;
    off = nq_of(l);
    nq = nq_of(l);
  }
  DevBuf rec;
  if (rec_stride && fbc_digit_path(T, *tab, nq)) {
    *rec_stride = (size_t)np * (per + 1) * N;
    rec = DevBuf(&pool, xs.size() * *rec_stride);
  }
  launch_intt_many(T, bases, np * per, per, x0.nlimbs, off, m, stream, rec.p ? tab : nullptr, rec.p);
  return rec;
}

HeCt HeCtxImpl::keyswitch(const u64* d, int level, u64 g_key, int B) {
  DevBuf dig = decompose(d, level, B);
  HeCt h = ct_new(level, true, 1.0, B);
  const DevBuf& k = key(g_key);
  launch_multsum(T, h.d.p, dig.p, k.p, nullptr, pmod.p, level, L, alpha, beta_at(level), 1, B, stream);
  n_multsum += B;
  return moddown(h, -1, true);
}

HeCt HeCtxImpl::mult(const HeCt& a, const HeCt& b) {
  need_same(a, b);
  if (a.packed || b.packed) fail(HE_EINVAL, "packed limbs are for the tensor sums alone");
  if (a.qp) fail(HE_EINVAL, "mult of R_QP elements");
  int nl = a.nlimbs, nt = a.B * nl;
  DevBuf t3(&pool, (size_t)3 * nt * N);
  launch_tensor(T, t3.p, a.d.p, b.d.p, nl, a.B, false, stream);
  HeCt ks = keyswitch(t3.p + (size_t)2 * nt * N, a.level, 0, a.B);
  HeCt c = ct_new(a.level, false, a.scale * b.scale, a.B);
  launch_add(T, c.d.p, t3.p, ks.d.p, 2 * nt, qmap(nl), stream);
  return c;
}

HeCt HeCtxImpl::rotate(const HeCt& x, long step) {
  if (x.packed) fail(HE_EINVAL, "packed limbs are for the tensor sums alone");
  u64 g = galois(step);
  if (g == 1) return ct_copy(x);
  DevBuf dig = decompose(x.poly(1), x.level, x.B);
  HeCt h = hoisted(x, dig.p, g);
  return moddown(h, -1, true);
}

// Rotations of a batch x (one level and scale) by several steps, hoisted
// (section 3.3.1): one Decompose of the whole batch, the key inner products
// of every step in one multi-rotation launch, one ModDown per step.  out[r]
// is x rotated by steps[r], with the residues rotate() gives.
std::vector<HeCt> HeCtxImpl::rotate_many(const HeCt& x, const std::vector<long>& steps) {
  if (x.qp) fail(HE_EINVAL, "rotation of an R_QP element");
  std::vector<HeCt> out(steps.size());
  std::vector<u64> gs;
  std::vector<size_t> where;
  for (size_t r = 0; r < steps.size(); r++) {
    const u64 g = galois(steps[r]);
    if (g == 1) {
      out[r] = ct_copy(x);
    } else {
      key(g);  // a missing key fails before anything is launched
      gs.push_back(g);
      where.push_back(r);
    }
  }
  if (gs.empty()) return out;
  DevBuf dig = decompose(x.poly(1), x.level, x.B);
  for (size_t r0 = 0; r0 < gs.size(); r0 += MR_MAX) {
    const size_t nr = std::min(gs.size() - r0, (size_t)MR_MAX);
    std::vector<HeCt> h = hoisted_multi(x, dig.p, std::vector<u64>(gs.begin() + r0, gs.begin() + r0 + nr));
    for (size_t r = 0; r < nr; r++) {
      out[where[r0 + r]] = moddown(h[r], -1, true);
      h[r] = HeCt();
    }
  }
  return out;
}

// device words a rotation of B members at `level` takes besides its input and
// output (Decompose's coefficients and digits, the R_{Q_l P} hoisted
// rotation, ModDown's special-prime limbs, lift and quotient), each block
// rounded up to the pool's 256-byte granule
size_t HeCtxImpl::rotate_workspace_bytes(int level, int B) const {
  const size_t nq = nq_of(level), nqp = nqp_of(level), bl = beta_at(level), np = 2 * (size_t)B;
  const size_t blocks[] = {B * nq, B * bl * nqp, np * nqp, np * alpha, np * nq, np * (alpha + 1)};
  size_t total = 0;
  for (size_t w : blocks) total += (w * N * 8 + 255) & ~(size_t)255;
  return total;
}

// Rotation into a caller's buffer with every temporary taken from `ws`
// (bytes of device memory): no pool block is requested.  The residues are
// those of rotate().
void HeCtxImpl::rotate_into(const HeCt& x, long step, u64* out, void* ws, size_t ws_bytes) {
  if (x.qp) fail(HE_EINVAL, "rotation of an R_QP element");
  const u64 g = galois(step);
  if (g == 1) {
    if (out != x.d.p)
      hip_check(hipMemcpyAsync(out, x.d.p, x.d.words * 8, hipMemcpyDeviceToDevice, stream), "copy");
    return;
  }
  if (rotate_workspace_bytes(x.level, x.B) > ws_bytes) fail(HE_EINVAL, "rotation needs a larger workspace");
  key(g);  // a missing key fails before anything is launched
  DevPool ws_pool;
  ws_pool.bump_base = (char*)ws;
  ws_pool.bump_cap = ws_bytes;
  DevPool* saved = pool.redirect;
  pool.redirect = &ws_pool;
  try {
    DevBuf dig = decompose(x.poly(1), x.level, x.B);
    HeCt h = hoisted(x, dig.p, g);
    moddown_to(h, x.level, out);
  } catch (...) {
    pool.redirect = saved;
    throw;
  }
  pool.redirect = saved;
}

HeCt HeCtxImpl::pmult_int(const HeCt& a, const i64* m_dev, double pt_scale) {
  LimbMap m = a.qp ? qpmap(a.level) : qmap(a.level + 1);
  DevBuf pt(&pool, (size_t)a.nlimbs * N);
  int_to_ntt(pt.p, m_dev, m);
  HeCt c = ct_new(a.level, a.qp, a.scale * pt_scale, a.B);
  launch_mul_bcast(T, c.d.p, a.d.p, pt.p, (int)a.polys() * a.nlimbs, a.nlimbs, m, stream);
  return c;
}

// B single ciphertexts of one level and scale -> one batch, and back
HeCt HeCtxImpl::stack(const std::vector<const HeCt*>& xs) {
  const HeCt& x0 = *xs[0];
  for (auto* x : xs)
    if (x->level != x0.level || x->qp || x->B != 1 || x->scale != x0.scale)
      fail(HE_EINVAL, "batched members must share level and scale");
  HeCt c = ct_new(x0.level, false, x0.scale, (int)xs.size());
  for (size_t b = 0; b < xs.size(); b++)
    for (int p = 0; p < 2; p++) copy_limbs(c.member(p, (int)b), xs[b]->poly(p), x0.nlimbs, "copy_stack");
  return c;
}
std::vector<HeCt> HeCtxImpl::unstack(const HeCt& x) {
  std::vector<HeCt> out;
  for (int b = 0; b < x.B; b++) {
    HeCt c = ct_new(x.level, x.qp, x.scale, 1);
    for (int p = 0; p < 2; p++) copy_limbs(c.poly(p), x.member(p, b), x.nlimbs, "copy_unstack");
    out.push_back(std::move(c));
  }
  return out;
}

// ---------------------------------------------------------------------------
// plaintext diagonals (cached per transform, level and basis)
// ---------------------------------------------------------------------------
// ensure every vector in `vecs` (each of length n2) has an evaluation-domain
// plaintext over Q_level (+P if qp) under cache key keys[i]; returns pointers
std::vector<const u64*> HeCtxImpl::plaintexts(const std::vector<std::string>& keys_, const PtGen& gen, int n2,
                                              int level, bool qp, double scale) {
  std::vector<const u64*> out(keys_.size(), nullptr);
  std::vector<int> missing;
  char suffix[96];
  snprintf(suffix, sizeof suffix, "|L%d|%d|%.17g", level, qp ? 1 : 0, scale);
  for (size_t i = 0; i < keys_.size(); i++) {
    auto it = ptcache.find(keys_[i] + suffix);
    if (it != ptcache.end()) out[i] = it->second.p;
    else missing.push_back((int)i);
  }
  if (missing.empty()) return out;
  LimbMap m = qp ? qpmap(level) : qmap(level + 1);
  int nl = m.n;
  const int chunk = std::max(1, (int)std::min<u64>(256, (1ull << 26) / N));
  for (size_t s0 = 0; s0 < missing.size(); s0 += chunk) {
    int b = (int)std::min(missing.size() - s0, (size_t)chunk);
    std::vector<double> host((size_t)b * n2), v;
    for (int t = 0; t < b; t++) {
      gen(missing[s0 + t], v);
      if ((int)v.size() != n2) fail(HE_EINVAL, "plaintext vector of the wrong length");
      std::copy(v.begin(), v.end(), host.begin() + (size_t)t * n2);
    }
    DevBuf ints = encode_batch(host.data(), n2, b, scale);
    for (int t = 0; t < b; t++) {
      int i = missing[s0 + t];
      DevBuf pt(&pool, (size_t)nl * N);
      int_to_ntt(pt.p, (const i64*)ints.p + (size_t)t * N, m);
      out[i] = pt.p;
      ptcache[keys_[i] + suffix] = std::move(pt);
    }
  }
  return out;
}

// ---------------------------------------------------------------------------
// Jiang's permutations (Eq. 4) on the row-major n^2 vector: output t takes
// input perm[t].
// ---------------------------------------------------------------------------
std::vector<int> make_perm(int kind, int n) {
  std::vector<int> p((size_t)n * n);
  for (int i = 0; i < n; i++)
    for (int j = 0; j < n; j++) {
      int t = i * n + j;
      if (kind == LT_SIGMA) p[t] = i * n + (i + j) % n;
      else if (kind == LT_TAU) p[t] = ((i + j) % n) * n + j;
      else p[t] = j * n + i;
    }
  return p;
}

static long pmod_l(long a, long m) { return ((a % m) + m) % m; }

// diagonal l of the (weighted) permutation, pre-rotated right by `shift`
// the 1-entries of a permutation grouped by diagonal: diagonal l (mod n^2)
// holds the positions s with perm[s] - s = l
using DiagGroups = std::unordered_map<long, std::vector<int>>;
static DiagGroups diag_groups(const std::vector<int>& perm) {
  const long n2 = (long)perm.size();
  DiagGroups g;
  for (long s = 0; s < n2; s++)
    if (perm[s] >= 0) g[pmod_l((long)perm[s] - s, n2)].push_back((int)s);
  return g;
}

// diagonal l of the permutation matrix rotated by `shift` slots, times w;
// false when that diagonal is empty
static bool diag_vec(const DiagGroups& groups, long n2, long l, long shift, double w, std::vector<double>& out) {
  auto it = groups.find(pmod_l(l, n2));
  if (it == groups.end()) return false;
  out.assign(n2, 0.0);
  for (int s : it->second) out[pmod_l(s + shift, n2)] = w;
  return true;
}

static int ceil_div_i(int a, int b) { return (a + b - 1) / b; }

LtGeom lt_geom(int kind, int n, int n1) {
  LtGeom g;
  g.n1 = n1;
  int n2 = ceil_div_i(n, n1);
  if (kind == LT_SIGMA) { g.a = 1; g.i_lo = -n2; g.i_hi = n2; }
  else if (kind == LT_TAU) { g.a = n; g.i_lo = 0; g.i_hi = n2; }
  else { g.a = n - 1; g.i_lo = -n2; g.i_hi = n2; }
  return g;
}

// double-hoisted BSGS: U x = sum_i rot( sum_j rot(u_{a(n1 i+j)}, -a n1 i) (.) rot(x, a j), a n1 i )
HeCt HeCtxImpl::lintrans(const HeCt& x, int kind, int n, int n1, double weight) {
  if ((u64)n * n > N / 2 || n1 < 1) fail(HE_EINVAL, "matrix does not fit the slots");
  char tag[64];
  snprintf(tag, sizeof tag, "lt%d|n%d", kind, n);
  return lintrans_perm(x, make_perm(kind, n), lt_geom(kind, n, n1), weight, tag);
}

// Z or T by double-hoisted BSGS with the simple key substitution of the
// baby steps (section 4.2.1): only the keys a j', j' < n1p, of the inner loop
HeCt HeCtxImpl::lintrans_smpkeysub(const HeCt& x, int kind, int n, int n1, int n1p) {
  if ((u64)n * n > N / 2 || n1 < 1) fail(HE_EINVAL, "matrix does not fit the slots");
  if (n1p == 1) fail(HE_EINVAL, "a prefix of one baby step holds no key to step with");
  char tag[64];
  snprintf(tag, sizeof tag, "lt%d|n%d", kind, n);
  return lintrans_perm(x, make_perm(kind, n), lt_geom(kind, n, n1), 1.0, tag, n1p);
}

// rotation steps a double-hoisted BSGS over `perm` with geometry G performs
// (with n1p as in lintrans_perm: baby steps from the prefix a j', j' < n1p)
void bsgs_steps(const std::vector<int>& perm, const LtGeom& G, std::set<long>& out, int n1p) {
  const DiagGroups groups = diag_groups(perm);
  const long n2 = (long)perm.size();
  const int m = (n1p >= 2 && n1p < G.n1) ? n1p : G.n1;
  for (int i = G.i_lo; i < G.i_hi; i++) {
    bool any = false;
    for (int j = 0; j < G.n1; j++) {
      long l = (long)G.a * ((long)G.n1 * i + j);
      if (!groups.count(pmod_l(l, n2))) continue;
      any = true;
      if (j % m) out.insert((long)G.a * (j % m));
    }
    if (any && i) out.insert((long)G.a * G.n1 * i);
  }
  if (m < G.n1) {
    // the blocks' bases: HR by a (m - 1), then Rot by a
    out.insert((long)G.a * (m - 1));
    out.insert((long)G.a);
  }
}

HeCt HeCtxImpl::lintrans_perm(const HeCt& x, const std::vector<int>& perm, const LtGeom& G, double weight,
                              const std::string& tag, int n1p) {
  if (x.qp) fail(HE_EINVAL, "linear transform of an R_QP element");
  if (x.level < 1) fail(HE_ELEVEL, "linear transform needs one level");
  const int n1 = G.n1;
  const int n2sq = (int)perm.size();
  const int level = x.level;
  const int nqp = nqp_of(level);
  // diagonals encoded at scale q_l: the closing rescale by q_l gives back
  // exactly the input scale
  const double ql = (double)mods[level];
  // the diagonals present and their plaintexts, found once per transform,
  // geometry, weight and level
  char plan_key[256];
  snprintf(plan_key, sizeof plan_key, "%s|a%ld|n1_%d|i%d..%d|w%.17g|L%d", tag.c_str(), (long)G.a, n1, G.i_lo,
           G.i_hi, weight, level);
  auto pit = ltplans.find(plan_key);
  if (pit == ltplans.end()) {
    const DiagGroups groups = diag_groups(perm);
    std::vector<std::string> keys_;
    std::vector<std::vector<double>> vecs;
    LtPlan plan;
    std::vector<double> v;
    for (int i = G.i_lo; i < G.i_hi; i++)
      for (int j = 0; j < n1; j++) {
        long l = (long)G.a * ((long)n1 * i + j);
        if (!diag_vec(groups, n2sq, l, (long)G.a * n1 * i, weight, v)) continue;
        char key[160];
        snprintf(key, sizeof key, "%s|a%ld|n1_%d|i%d|j%d|w%.17g", tag.c_str(), (long)G.a, n1, i, j, weight);
        keys_.push_back(key);
        vecs.push_back(v);
        plan.ij.push_back({i, j});
      }
    if (plan.ij.empty()) fail(HE_EINVAL, "transform has no nonzero diagonal");
    plan.pts = plaintexts(keys_, [&](size_t e, std::vector<double>& o) { o = vecs[e]; }, n2sq, level, true, ql);
    pit = ltplans.emplace(plan_key, std::move(plan)).first;
  }
  const std::vector<std::pair<int, int>>& ij = pit->second.ij;
  const std::vector<const u64*>& pts = pit->second.pts;
  std::vector<bool> used(n1, false);
  for (auto& p : ij) used[p.second] = true;
  // Decompose once, baby-step hoisted rotations kept in R_{Q_l P}.  With the
  // simple key substitution (section 4.2.1, 2 <= n1p < n1) the baby steps
  // a (b n1p + j') come in blocks of n1p, each hoisted from its own base
  // x_b = Rot(x_{b-1}, a n1p) with the prefix keys a j' (j' < n1p): x_b is
  // the ModDown of the block before's last hoisted rotation
  // HR(x_{b-1}, a (n1p - 1)), rotated once more by a.
  const int m = (n1p >= 2 && n1p < n1) ? n1p : n1;
  std::vector<HeCt> baby(n1);
  HeCt xb;
  for (int b = 0; b * m < n1; b++) {
    const HeCt& base = b == 0 ? x : xb;
    const bool more = (b + 1) * m < n1;
    const int jl = b * m + m - 1;
    std::vector<u64> gs;
    std::vector<int> js;
    for (int jp = 0; jp < m && b * m + jp < n1; jp++)
      if (used[b * m + jp] || (more && jp == m - 1)) {
        gs.push_back(galois((long)G.a * jp));
        js.push_back(b * m + jp);
      }
    {
      DevBuf dig = decompose(base.poly(1), level, base.B);
      std::vector<HeCt> hs = hoisted_multi(base, dig.p, gs);
      for (size_t t = 0; t < js.size(); t++) baby[js[t]] = std::move(hs[t]);
    }
    if (more) {
      HeCt y = moddown(baby[jl]);
      if (!used[jl]) baby[jl] = HeCt();
      xb = rotate(y, G.a);
    }
  }
  xb = HeCt();
  LimbMap qpm = qpmap(level);
  HeCt acc = ct_new(level, true, x.scale * ql, x.B);
  bool acc_set = false;
  // giant steps with at least one diagonal: (j, index into pts) per step
  std::map<int, std::vector<std::pair<int, size_t>>> by_i;
  for (size_t e = 0; e < ij.size(); e++) by_i[ij[e].first].push_back({ij[e].second, e});
  std::vector<int> gi;
  for (auto& kv : by_i) gi.push_back(kv.first);
  const int nl = 2 * x.B * nqp;
  for (size_t c0 = 0; c0 < gi.size(); c0 += SUM_MAX_OUTS) {
    const int ng = (int)std::min<size_t>(SUM_MAX_OUTS, gi.size() - c0);
    // inner_i = sum_j baby_j (.) diagonal_(i,j) for ng giant steps in one pass over the babies
    std::vector<int> col(n1, -1), jl;
    for (int g = 0; g < ng; g++)
      for (auto& je : by_i[gi[c0 + g]])
        if (col[je.first] < 0) {
          col[je.first] = (int)jl.size();
          jl.push_back(je.first);
        }
    const int nt = (int)jl.size();
    std::vector<const u64*> ta(nt), tp((size_t)ng * nt, nullptr);
    for (int t = 0; t < nt; t++) ta[t] = baby[jl[t]].d.p;
    std::vector<HeCt> inner(ng);
    std::vector<u64*> outs(ng);
    for (int g = 0; g < ng; g++) {
      for (auto& je : by_i[gi[c0 + g]]) tp[(size_t)g * nt + col[je.first]] = pts[je.second];
      inner[g] = ct_new(level, true, x.scale * ql, x.B);
      outs[g] = inner[g].d.p;
    }
    if (!launch_mul_sum_multi(T, outs.data(), ng, ta.data(), tp.data(), nt, nl, nqp, qpm, stream)) {
      for (int g = 0; g < ng; g++) {
        std::vector<const u64*> a1, p1;
        for (int t = 0; t < nt; t++)
          if (tp[(size_t)g * nt + t]) {
            a1.push_back(ta[t]);
            p1.push_back(tp[(size_t)g * nt + t]);
          }
        launch_mul_sum(T, outs[g], a1.data(), p1.data(), (int)a1.size(), nl, nqp, qpm, false, stream);
      }
    }
    for (int g = 0; g < ng; g++) {
      const int i = gi[c0 + g];
      HeCt term;
      if (i == 0) {
        term = std::move(inner[g]);
      } else {
        HeCt t = moddown(inner[g], -1, true);
        inner[g] = HeCt();
        DevBuf d2 = decompose(t.poly(1), level, t.B);
        term = hoisted(t, d2.p, galois((long)G.a * n1 * i));
      }
      if (!acc_set) {
        acc = std::move(term);
        acc_set = true;
      } else {
        add_into(acc, term);
      }
    }
  }
  HeCt md = moddown(acc, -1, true);
  HeCt r = rescale(md);
  r.scale = x.scale;
  return r;
}

// ---------------------------------------------------------------------------
// The matrix product (Eq. 4; Algorithm DMatrixMult; hoisted C^k / R^k of
// section 4.1.1)
// ---------------------------------------------------------------------------
int default_n1(int n) {
  int lg = 0;
  while ((1 << lg) < n) lg++;
  return 1 << ((lg + 1) / 2);
}

// ---------------------------------------------------------------------------
// Diagonal convergence decomposition (section 4.2: Definition 4, Theorem 2,
// Algorithms DCDforZ / DCDforT).  Each 1-entry of the permutation with
// remaining diagonal k is moved by the right factors one step r(k) at a time
// (same column, Definition 4); the left factor takes what remains.
//   Z (split into k >= 0 and k < 0): r = sign(k) n' while |k| >= n'
//   T (k = i n):                      r = n' n     while i > n'
// ---------------------------------------------------------------------------
static long floor_div_l(long a, long b) { return a >= 0 ? a / b : -((-a + b - 1) / b); }

std::vector<DcdFactor> dcd_chain(int n, const std::vector<int>& perm, int which, int nprime, int n1) {
  const int n2 = n * n;
  const int iters = ceil_div_i(n - 1, nprime) - 1;
  std::vector<long> pos(n2, -1), rem(n2, 0);
  std::vector<char> sel(n2, 0);
  for (int t = 0; t < n2; t++) {
    long k = which == DCD_T ? pmod_l((long)perm[t] - t, n2) : (long)perm[t] - t;
    if ((which == DCD_Z1 && k < 0) || (which == DCD_Z2 && k >= 0)) continue;
    sel[t] = 1;
    pos[t] = perm[t];
    rem[t] = k;
  }
  const long step = which == DCD_Z1 ? nprime : which == DCD_Z2 ? -(long)nprime : (long)nprime * n;
  std::vector<DcdFactor> out;
  for (int it = 0; it < iters; it++) {
    DcdFactor f;
    f.perm.assign(n2, -1);
    for (int t = 0; t < n2; t++) {
      if (!sel[t]) continue;
      long r = which == DCD_T ? (rem[t] / n > nprime ? step : 0) : (std::labs(rem[t]) >= nprime ? step : 0);
      long np = pmod_l(pos[t] - r, n2);
      if (f.perm[np] != -1) fail(HE_EINVAL, "decomposition factor is not a partial permutation");
      f.perm[np] = (int)pos[t];
      pos[t] = np;
      rem[t] -= r;
    }
    f.G = LtGeom{(int)step, 2, 0, 1};
    out.push_back(std::move(f));
  }
  DcdFactor lf;
  lf.perm.assign(n2, -1);
  const long a = which == DCD_T ? n : 1;
  long kmin = 0, kmax = 0;
  bool first = true;
  for (int t = 0; t < n2; t++) {
    if (!sel[t]) continue;
    lf.perm[t] = (int)pos[t];
    long kk = rem[t] / a;
    if (first || kk < kmin) kmin = kk;
    if (first || kk > kmax) kmax = kk;
    first = false;
  }
  lf.G = LtGeom{(int)a, n1, (int)floor_div_l(kmin, n1), (int)floor_div_l(kmax, n1) + 1};
  out.push_back(std::move(lf));
  return out;
}

void lintrans_steps(int kind, int n, int n1, int nprime, std::set<long>& s) {
  if (kind == LT_TRANSPOSE || nprime >= n - 1) {
    bsgs_steps(make_perm(kind, n), lt_geom(kind, n, n1), s);
    return;
  }
  std::vector<int> perm = make_perm(kind, n);
  std::vector<int> chains = kind == LT_SIGMA ? std::vector<int>{DCD_Z1, DCD_Z2} : std::vector<int>{DCD_T};
  for (int ch : chains)
    for (auto& f : dcd_chain(n, perm, ch, nprime, n1)) bsgs_steps(f.perm, f.G, s);
}

std::vector<long> matmul_steps(int n, int n1z, int n1t, int npz, int npt, bool folded) {
  std::set<long> s;
  lintrans_steps(LT_SIGMA, n, n1z, npz, s);
  lintrans_steps(LT_TAU, n, n1t, npt, s);
  // column shifts (r < n1z, chain n1z, second chain from -n; none when they
  // are folded into Z), row shifts (n r, chain n n1t)
  if (!folded) {
    for (int j = 1; j < n1z; j++) s.insert(j);
    s.insert(n1z);
    s.insert(-(long)n);
  }
  for (int j = 1; j < n1t; j++) s.insert((long)n * j);
  s.insert((long)n * n1t);
  return std::vector<long>(s.begin(), s.end());
}

std::vector<long> transpose_steps(int n, int n1) {
  std::set<long> s;
  lintrans_steps(LT_TRANSPOSE, n, n1, n - 1, s);
  return std::vector<long>(s.begin(), s.end());
}

HeCt HeCtxImpl::apply_chain(const HeCt& x, const std::vector<DcdFactor>& fs, const std::string& tag) {
  if (fs.empty()) return ct_copy(x);
  HeCt cur = lintrans_perm(x, fs[0].perm, fs[0].G, 1.0, tag + "|f0");
  for (size_t j = 1; j < fs.size(); j++) cur = lintrans_perm(cur, fs[j].perm, fs[j].G, 1.0, tag + "|f" + std::to_string(j));
  return cur;
}

// Z a: one double-hoisted BSGS, or the Z1 and Z2 chains of the decomposition
HeCt HeCtxImpl::sigma_dcd(const HeCt& x, int n, int n1, int nprime) {
  if (nprime >= n - 1) return lintrans(x, LT_SIGMA, n, n1, 1.0);
  std::vector<int> perm = make_perm(LT_SIGMA, n);
  char tag[64];
  snprintf(tag, sizeof tag, "dcdZ|n%d|np%d", n, nprime);
  HeCt a1 = apply_chain(x, dcd_chain(n, perm, DCD_Z1, nprime, n1), std::string(tag) + "|1");
  HeCt a2 = apply_chain(x, dcd_chain(n, perm, DCD_Z2, nprime, n1), std::string(tag) + "|2");
  return add(a1, a2, false);
}

HeCt HeCtxImpl::tau_dcd(const HeCt& x, int n, int n1, int nprime) {
  if (nprime >= n - 1) return lintrans(x, LT_TAU, n, n1, 1.0);
  char tag[64];
  snprintf(tag, sizeof tag, "dcdT|n%d|np%d", n, nprime);
  return apply_chain(x, dcd_chain(n, make_perm(LT_TAU, n), DCD_T, nprime, n1), tag);
}

static void col_mask(int n, int k, bool second, std::vector<double>& out) {
  out.assign((size_t)n * n, 0.0);
  for (int i = 0; i < n; i++)
    for (int j = 0; j < n; j++) {
      bool first = j < n - k;
      out[(size_t)i * n + j] = (second ? !first : first) ? 1.0 : 0.0;
    }
}

// A side: A_k = C^k Z a.  A_k = Rescale(ModDown(m_k (.) HR(B_b, r) + m'_k (.) HR(B'_b, r))),
// k = b n1z + r, with bases B_b = Rot(B_{b-1}, n1z), B'_0 = Rot(Z a, -n), B'_b = Rot(B'_{b-1}, n1z)
// out_level (if >= 0) caps the level of the A_k: limbs above it are never
// computed (the same residues as computing them and dropping them).
std::vector<HeCt> HeCtxImpl::matmul_side_a(const HeCt& ca, int n, int n1z, int npz, int out_level, bool fused_rs,
                                           bool pack) {
  HeCt A0 = sigma_dcd(ca, n, n1z, npz);
  const int lvl = A0.level;
  if (lvl < 1) fail(HE_ELEVEL, "no level left for the column shifts");
  const int nqp = nqp_of(lvl);
  LimbMap qpm = qpmap(lvl);
  std::vector<std::string> keys_;
  std::vector<std::pair<int, int>> which;
  for (int k = 0; k < n; k++) {
    for (int second = 0; second < 2; second++) {
      if (second && k == 0) continue;
      char key[64];
      snprintf(key, sizeof key, "colmask|n%d|k%d|%d", n, k, second);
      keys_.push_back(key);
      which.push_back({k, second});
    }
  }
  // masks encoded at scale q_lvl: each rescale restores the base's scale
  const double ql = (double)mods[lvl];
  std::vector<const u64*> masks = plaintexts(
      keys_, [&](size_t e, std::vector<double>& o) { col_mask(n, which[e].first, which[e].second != 0, o); }, n * n,
      lvl, true, ql);
  auto mask_of = [&](int k, int second) { return masks[k == 0 ? 0 : 2 * k - 1 + second]; };
  std::vector<HeCt> Ak(n);
  HeCt Bb = ct_copy(A0), Bpb = rotate(A0, -(long)n);
  A0 = HeCt();
  for (int b = 0; b * n1z < n; b++) {
    if (b > 0) {
      Bb = rotate(Bb, n1z);
      Bpb = rotate(Bpb, n1z);
    }
    // all n1z hoisted rotations of each base in one launch per base; the
    // masks are applied in the launch's epilogue, the second base's masked
    // rotations added onto the first's, so that the hoisted rotations
    // themselves never reach memory.  r = 0 (Galois element 1) is the P-lift.
    const int nr = std::min(n1z, n - b * n1z);
    std::vector<HeCt> acc(nr);
    for (int r = 0; r < nr; r++) acc[r] = ct_new(lvl, true, Bb.scale * ql, Bb.B);
    std::vector<u64> gs;
    std::vector<u64*> outs;
    std::vector<const u64*> m1, m2;
    for (int r = 1; r < nr; r++) {
      const int k = b * n1z + r;
      gs.push_back(galois(r));
      outs.push_back(acc[r].d.p);
      m1.push_back(mask_of(k, 0));
      m2.push_back(mask_of(k, 1));
    }
    HeCt lift1, lift2;
    {
      // both bases' masked rotations in one launch where it applies (each
      // key word loaded once), else the second added onto the first
      DevBuf d1 = decompose(Bb.poly(1), lvl, Bb.B);
      DevBuf d2 = decompose(Bpb.poly(1), lvl, Bpb.B);
      if (!hoisted_masked_pair(Bb, d1.p, m1, Bpb, d2.p, m2, gs, outs)) {
        hoisted_masked(Bb, d1.p, gs, outs, m1, false);
        hoisted_masked(Bpb, d2.p, gs, outs, m2, true);
      }
      lift1 = hoisted(Bb, d1.p, 1);
      if (b > 0) lift2 = hoisted(Bpb, d2.p, 1);  // k = 0 has no second term
    }
    {
      // r = 0: the P-lifts times their masks
      const int k = b * n1z;
      const u64* ta[2] = {lift1.d.p, k > 0 ? lift2.d.p : nullptr};
      const u64* tp[2] = {mask_of(k, 0), mask_of(k, 1)};
      launch_mul_sum(T, acc[0].d.p, ta, tp, k > 0 ? 2 : 1, 2 * Bb.B * nqp, nqp, qpm, false, stream);
      lift1 = HeCt();
      lift2 = HeCt();
    }
    DevBuf rec;
    size_t rs = 0;
    {
      std::vector<HeCt*> srcs;
      for (auto& a : acc) srcs.push_back(&a);
      rec = moddown_sources(srcs, fused_rs, &rs);
    }
    const bool ready = fused_conv;
    for (int r = 0; r < nr; r++) {
      int k = b * n1z + r;
      HeCt sum = std::move(acc[r]);
      const int ol = out_level >= 0 ? std::min(out_level, lvl - 1) : -1;
      const u64* rr = rec.p ? rec.p + r * rs : nullptr;
      if (fused_rs) {
        Ak[k] = moddown_rescale(sum, ol, true, ready, rr, pack);
      } else {
        HeCt md = moddown(sum, -1, true, ready, rr);
        Ak[k] = rescale(md, ol);
      }
      Ak[k].scale = Bb.scale;
    }
  }
  return Ak;
}

// B side: B_k = R^k T b.  C_0 = T b, C_b = Rot(C_{b-1}, n n1t), B_k = ModDown(HR(C_b, n r))
// out_level (if >= 0) caps the level of the B_k, as for the A side
std::vector<HeCt> HeCtxImpl::matmul_side_b(const HeCt& cb, int n, int n1t, int npt, int out_level, bool pack) {
  HeCt Cb = tau_dcd(cb, n, n1t, npt);
  const int lvl = Cb.level;
  const int ol = out_level >= 0 ? std::min(out_level, lvl) : lvl;
  std::vector<HeCt> Bk(n);
  for (int b = 0; b * n1t < n; b++) {
    if (b > 0) Cb = rotate(Cb, (long)n * n1t);
    const int nr = std::min(n1t, n - b * n1t);
    std::vector<HeCt> hs;
    {
      DevBuf d1 = decompose(Cb.poly(1), lvl, Cb.B);
      std::vector<u64> gs;
      for (int r = 1; r < nr; r++) gs.push_back(galois((long)n * r));
      hs = hoisted_multi(Cb, d1.p, gs);
    }
    Bk[b * n1t] = ol < lvl ? drop(Cb, ol) : ct_copy(Cb);
    DevBuf rec;
    size_t rs = 0;
    {
      std::vector<HeCt*> srcs;
      for (auto& h : hs) srcs.push_back(&h);
      rec = moddown_sources(srcs, false, &rs);
    }
    for (int r = 1; r < nr; r++) {
      Bk[b * n1t + r] = moddown(hs[r - 1], ol, true, fused_conv, rec.p ? rec.p + (r - 1) * rs : nullptr, pack);
      hs[r - 1] = HeCt();
    }
  }
  return Bk;
}

// A side with the masks of C^k folded into Z: phi^k o sigma (output (i, j)
// takes A_{i, (i + j + k) mod n}) is a permutation whose diagonals are C^k's
// masks times Z's diagonals, at Z's diagonal indices, so A_k is one
// double-hoisted BSGS transform of a with Z's geometry and keys: one level
// where section 4.1.1's masked shifts add a second.
std::vector<HeCt> HeCtxImpl::matmul_side_a_folded(const HeCt& ca, int n, int n1z) {
  std::vector<HeCt> Ak(n);
  const LtGeom G = lt_geom(LT_SIGMA, n, n1z);
  std::vector<int> perm((size_t)n * n);
  for (int k = 0; k < n; k++) {
    for (int i = 0; i < n; i++)
      for (int j = 0; j < n; j++) perm[(size_t)i * n + j] = i * n + (i + j + k) % n;
    char tag[64];
    snprintf(tag, sizeof tag, "foldZ|n%d|k%d", n, k);
    Ak[k] = lintrans_perm(ca, perm, G, 1.0, tag);
  }
  return Ak;
}

// drop both sides to their common (lowest) level
void HeCtxImpl::align_sides(std::vector<HeCt>& Ak, std::vector<HeCt>& Bk) {
  int lv = std::min(Ak[0].level, Bk[0].level);
  for (auto& a : Ak)
    if (a.level > lv) a = drop(a, lv);
  for (auto& b : Bk)
    if (b.level > lv) b = drop(b, lv);
}

// acc (+)= sum_k Relin(Tensor(A_k, B_k))
void HeCtxImpl::matmul_accumulate(HeCt& acc, bool& acc_set, const std::vector<HeCt>& Ak, const std::vector<HeCt>& Bk) {
  for (size_t k = 0; k < Ak.size(); k++) {
    HeCt p = mult(Ak[k], Bk[k]);
    if (!acc_set) {
      acc = std::move(p);
      acc_set = true;
    } else {
      add_into(acc, p);
    }
  }
}

// Lazy relinearisation (a variant of the paper's order): the tensors of
// all products are summed in three components, [3][B][nl][N] ...
void HeCtxImpl::accumulate_tensors(DevBuf& acc3, bool& acc_set, const std::vector<HeCt>& Ak,
                                   const std::vector<HeCt>& Bk) {
  const HeCt& a0 = Ak[0];
  const int nl = a0.nlimbs;
  if (!acc_set) acc3 = DevBuf(&pool, (size_t)3 * a0.B * nl * N);
  std::vector<const u64*> pa, pb;
  std::unique_ptr<bool[]> ka(new bool[Ak.size()]), kb(new bool[Ak.size()]);
  for (size_t k = 0; k < Ak.size(); k++) {
    need_same(Ak[k], Bk[k]);
    need_same(Ak[k], a0);
    pa.push_back(Ak[k].d.p);
    pb.push_back(Bk[k].d.p);
    ka[k] = Ak[k].packed;
    kb[k] = Bk[k].packed;
  }
  launch_tensor_sum(T, acc3.p, pa.data(), pb.data(), (int)pa.size(), nl, a0.B, acc_set, stream, ka.get(), kb.get());
  acc_set = true;
}
// ... and relinearised once
HeCt HeCtxImpl::relin_sum(const DevBuf& acc3, int level, double scale, int B) {
  const int nl = level + 1, nt = B * nl;
  HeCt ks = keyswitch(acc3.p + (size_t)2 * nt * N, level, 0, B);
  HeCt c = ct_new(level, false, scale, B);
  launch_add(T, c.d.p, acc3.p, ks.d.p, 2 * nt, qmap(nl), stream);
  return c;
}

HeCt HeCtxImpl::matmul(const HeCt& ca, const HeCt& cb, int n, int n1z, int n1t, int npz, int npt, bool lazy,
                        bool fused_rs, bool folded) {
  if (ca.qp || cb.qp || ca.level != cb.level) fail(HE_ELEVEL, "operands must be ciphertexts at one level");
  if ((u64)n * n > N / 2 || n % n1z || n % n1t || npz < 1 || npt < 1)
    fail(HE_EINVAL, "bad matrix size / baby-step count / decomposition");
  if (folded && (fused_rs || npz < n - 1))
    fail(HE_EINVAL, "the folded A side takes neither a decomposition of Z nor one rounding");
  int dz = npz >= n - 1 ? 1 : ceil_div_i(n - 1, npz), dt = npt >= n - 1 ? 1 : ceil_div_i(n - 1, npt);
  // A side: Z (dz levels), then the masked shifts (one level), or both in one
  // transform when folded
  const int da = folded ? 1 : dz + 1;
  if (ca.level < std::max(da, dt) + 1) fail(HE_ELEVEL, "not enough levels for the product");
  // both sides produced at their common level (A: sigma, then the masks;
  // B: tau); align_sides only guards the prediction
  const int common = std::min(ca.level - da, cb.level - dt);
  // the sides come out packed where only the lazy tensor sums read them
  std::vector<HeCt> Ak =
      folded ? matmul_side_a_folded(ca, n, n1z) : matmul_side_a(ca, n, n1z, npz, common, fused_rs, lazy);
  std::vector<HeCt> Bk = matmul_side_b(cb, n, n1t, npt, common, lazy);
  align_sides(Ak, Bk);
  HeCt acc;
  if (lazy) {
    DevBuf acc3;
    bool set = false;
    accumulate_tensors(acc3, set, Ak, Bk);
    acc = relin_sum(acc3, Ak[0].level, Ak[0].scale * Bk[0].scale, Ak[0].B);
  } else {
    bool set = false;
    matmul_accumulate(acc, set, Ak, Bk);
  }
  return rescale(acc);
}

// Recording: one eager run fills every cache (plaintext diagonals, tables);
// a second run inside the graph's arena (exact-size blocks) sizes it; the
// third, inside a stream capture, finds every block it asks for in the arena
// (frozen: no device allocation can happen during the capture).  A replay
// reads the operands' buffers as they are at that time and rewrites the
// arena's outputs, which are then copied out.
std::vector<HeCt> HeCtxImpl::matmul_graph(const std::vector<const HeCt*>& a, const std::vector<const HeCt*>& b,
                                          int n, int n1z, int n1t, int npz, int npt, bool lazy, bool fused_rs,
                                          bool folded) {
  if (a.empty() || a.size() != b.size() || a.size() > 8) fail(HE_EINVAL, "a recorded product takes 1 to 8 pairs");
  std::vector<u64> key{(u64)n,    (u64)n1z,      (u64)n1t,    (u64)npz,     (u64)npt,
                       (u64)lazy, (u64)fused_rs, (u64)folded, (u64)a.size()};
  for (const auto* v : {&a, &b})
    for (const HeCt* x : *v) {
      u64 sc;
      std::memcpy(&sc, &x->scale, 8);
      key.insert(key.end(), {(u64)(uintptr_t)x->d.p, (u64)x->level, sc, (u64)x->nlimbs, (u64)x->B});
    }
  auto it = graphs.begin();
  while (it != graphs.end() && it->key != key) ++it;
  if (it != graphs.end()) {
    graphs.splice(graphs.begin(), graphs, it);
  } else {
    if (graphs.size() >= 4) {
      // the evicted recording may still be replaying, and the copies out of
      // its arena may still be in flight
      hip_check(hipStreamSynchronize(stream), "graph eviction");
      graphs.pop_back();
    }
    auto run = [&](std::vector<HeCt>* keep) {
      HeCt sa = stack(a), sb = stack(b);
      HeCt r = matmul(sa, sb, n, n1z, n1t, npz, npt, lazy, fused_rs, folded);
      std::vector<HeCt> parts = unstack(r);
      if (keep) *keep = std::move(parts);
    };
    run(nullptr);
    graphs.emplace_front();
    MmGraph& g = graphs.front();
    g.key = key;
    g.arena.reset(new DevPool);
    g.arena->user_alloc = pool.user_alloc;
    g.arena->user_release = pool.user_release;
    g.arena->user = pool.user;
    g.arena->exact = true;
    g.arena->stream = stream;
    pool.redirect = g.arena.get();
    try {
      run(nullptr);
      hip_check(hipStreamSynchronize(stream), "graph arena");
      g.arena->frozen = true;
      hip_check(hipStreamBeginCapture(stream, hipStreamCaptureModeRelaxed), "begin capture");
      try {
        run(&g.outs);
      } catch (...) {
        hipGraph_t junk = nullptr;
        (void)hipStreamEndCapture(stream, &junk);
        if (junk) (void)hipGraphDestroy(junk);
        throw;
      }
      hip_check(hipStreamEndCapture(stream, &g.graph), "end capture");
      hip_check(hipGraphInstantiate(&g.exec, g.graph, nullptr, nullptr, 0), "graph instantiate");
    } catch (...) {
      pool.redirect = nullptr;
      g.outs.clear();
      graphs.pop_front();
      throw;
    }
    pool.redirect = nullptr;
    for (HeCt& o : g.outs) o.d.pool = g.arena.get();
  }
  MmGraph& g = graphs.front();
  hip_check(hipGraphLaunch(g.exec, stream), "graph launch");
  std::vector<HeCt> out;
  for (const HeCt& o : g.outs) out.push_back(ct_copy(o));
  return out;
}

namespace {
struct KsGroup {
  std::mutex mu;  // held by the job that is running
  std::condition_variable cv;
  int active = 0, waiting = 0;
  u64 generation = 0;
  bool failed = false;
  std::string error;
  std::vector<KsWork> pending;
};
}  // namespace

std::vector<HeCt> HeCtxImpl::run_merged(const std::vector<std::function<HeCt()>>& jobs) {
  KsGroup g;
  g.active = (int)jobs.size();
  std::vector<HeCt> res(jobs.size());
  std::vector<std::exception_ptr> errs(jobs.size());
  // with g.mu held: launch what is pending and release the waiting jobs
  auto flush = [&]() {
    if (!g.pending.empty() && !g.failed) {
      try {
        DevBuf tab(&pool, (multsum_list_table_bytes(T, g.pending, L, alpha) + 7) / 8);
        launch_multsum_list(T, g.pending, tab.p, tab.words * 8, L, alpha, stream);
      } catch (const HeError& e) {
        g.failed = true;
        g.error = e.msg;
      } catch (const std::exception& e) {
        g.failed = true;
        g.error = e.what();
      }
    }
    g.pending.clear();
    g.waiting = 0;
    g.generation++;
    g.cv.notify_all();
  };
  auto worker = [&](size_t t) {
    std::unique_lock<std::mutex> lk(g.mu);
    KsSink sink = [&](KsWork&& w) {
      if (g.failed) fail(HE_EDEVICE, "merged key switch failed: " + g.error);
      g.pending.push_back(std::move(w));
      g.waiting++;
      const u64 gen = g.generation;
      if (g.waiting == g.active) flush();
      else g.cv.wait(lk, [&] { return g.generation != gen; });
      if (g.failed) fail(HE_EDEVICE, "merged key switch failed: " + g.error);
    };
    KsSink* prev = ks_sink_exchange(&sink);
    try {
      res[t] = jobs[t]();
    } catch (...) {
      errs[t] = std::current_exception();
    }
    ks_sink_exchange(prev);
    g.active--;
    if (g.active > 0 && g.waiting == g.active) flush();
  };
  std::vector<std::thread> threads;
  for (size_t t = 0; t < jobs.size(); t++) threads.emplace_back(worker, t);
  for (auto& th : threads) th.join();
  for (auto& e : errs)
    if (e) std::rethrow_exception(e);
  return res;
}

void HeCtxImpl::drop_graphs() {
  if (graphs.empty()) return;
  (void)hipStreamSynchronize(stream);
  graphs.clear();
}

// Covariance (Algorithm HCovMtrx, centred data): block (a, b) of X^T X / s is
//   Rescale( sum_r sum_k Relin(Tensor(A_k(G(X_a[r]) / s), B_k(X_b[r]))) )
// for b <= a, and G(block (b, a)) for a < b; the A and B sides of each
// row block are formed once and reused for every pair (one-to-many caching).
CovState HeCtxImpl::cov_begin(int k, int n, u64 n_samples, int n1z, int n1t, int n1g, int npz, int npt, bool lazy,
                              bool fused_rs) {
  if (k < 1 || n < 2 || n_samples == 0) fail(HE_EINVAL, "bad covariance shape");
  CovState st;
  st.k = k;
  st.n = n;
  st.n_samples = n_samples;
  st.n1z = n1z;
  st.n1t = n1t;
  st.n1g = n1g;
  st.npz = npz;
  st.npt = npt;
  st.lazy = lazy;
  st.fused = fused_rs;
  st.acc.resize(k * k);
  st.acc3.resize(k * k);
  st.set.assign(k * k, false);
  return st;
}

void HeCtxImpl::cov_add(CovState& st, const std::vector<const HeCt*>& x, int rb) {
  const int k = st.k, n = st.n;
  if (rb < 1 || (int)x.size() != rb * k) fail(HE_EINVAL, "block count mismatch");
  const int level = x[0]->level;
  for (auto* c : x)
    if (c->level != level || c->qp) fail(HE_ELEVEL, "dataset blocks must share one level");
  if (st.level >= 0 && level != st.level) fail(HE_ELEVEL, "dataset blocks must share one level over all calls");
  const int dz = st.npz >= n - 1 ? 1 : ceil_div_i(n - 1, st.npz), dt = st.npt >= n - 1 ? 1 : ceil_div_i(n - 1, st.npt);
  if (level < std::max(dz + 1, dt) + 3) fail(HE_ELEVEL, "not enough levels for the covariance");
  st.level = level;
  // the sides' common level: A after the transposition, sigma and the masks,
  // B after tau
  const int common = std::min(level - 1 - dz - 1, level - 1 - dt);
  // row blocks go through the transforms and sides stacked, g at a time (a
  // batch of g members); each pair's products are summed over the members
  // into one accumulator (exact sums, so the residues depend neither on g
  // nor on how the row blocks are split over calls)
  int g = 4;
  knob_get("cov_row_blocks", &g);
  for (int r0 = 0; r0 < rb; r0 += g) {
    const int gb = std::min(g, rb - r0);
    auto rows_of = [&](int col) {
      std::vector<const HeCt*> xs;
      for (int r = r0; r < r0 + gb; r++) xs.push_back(x[r * k + col]);
      return gb == 1 ? ct_copy(*xs[0]) : stack(xs);
    };
    std::vector<std::vector<HeCt>> A(k), B(k);
    for (int a = 0; a < k; a++) {
      HeCt xt = lintrans(rows_of(a), LT_TRANSPOSE, n, st.n1g, 1.0 / (double)st.n_samples);
      A[a] = matmul_side_a(xt, n, st.n1z, st.npz, common, st.fused, st.lazy);
    }
    for (int b = 0; b < k; b++) {
      HeCt xb = drop(rows_of(b), level - 1);
      B[b] = matmul_side_b(xb, n, st.n1t, st.npt, common, st.lazy);
    }
    for (int a = 0; a < k; a++) align_sides(A[a], B[0]);
    for (int b = 0; b < k; b++) align_sides(A[0], B[b]);
    st.acc_level = A[0][0].level;
    st.acc_scale = A[0][0].scale * B[0][0].scale;
    const int nl = A[0][0].nlimbs;
    const LimbMap qm = qmap(nl);
    for (int a = 0; a < k; a++)
      for (int b = 0; b <= a; b++) {
        const int p = a * k + b;
        if (st.lazy) {
          DevBuf g3;
          bool gs = false;
          accumulate_tensors(g3, gs, A[a], B[b]);
          // [3][gb][nl][N] summed over the members into [3][1][nl][N]
          const size_t nt = (size_t)gb * nl;
          int m0 = 0;
          if (!st.set[p]) {
            st.acc3[p] = DevBuf(&pool, (size_t)3 * nl * N);
            for (int c = 0; c < 3; c++) copy_limbs(st.acc3[p].p + (size_t)c * nl * N, g3.p + c * nt * N, nl);
            m0 = 1;
            st.set[p] = true;
          }
          for (int c = 0; c < 3; c++)
            for (int m = m0; m < gb; m++) {
              u64* dst = st.acc3[p].p + (size_t)c * nl * N;
              launch_add(T, dst, dst, g3.p + (c * nt + (size_t)m * nl) * N, nl, qm, stream);
            }
        } else {
          HeCt gacc;
          bool gs = false;
          matmul_accumulate(gacc, gs, A[a], B[b]);
          std::vector<HeCt> parts = gb == 1 ? std::vector<HeCt>{} : unstack(gacc);
          if (gb == 1) parts.push_back(std::move(gacc));
          for (auto& part : parts) {
            if (!st.set[p]) {
              st.acc[p] = std::move(part);
              st.set[p] = true;
            } else {
              add_into(st.acc[p], part);
            }
          }
        }
      }
  }
  st.row_blocks += rb;
}

std::vector<HeCt> HeCtxImpl::cov_end(CovState& st) {
  const int k = st.k, n = st.n;
  if (st.row_blocks == 0) fail(HE_EINVAL, "covariance of no row blocks");
  std::vector<HeCt> out(k * k);
  for (int a = 0; a < k; a++)
    for (int b = 0; b <= a; b++) {
      if (st.lazy) {
        st.acc[a * k + b] = relin_sum(st.acc3[a * k + b], st.acc_level, st.acc_scale, 1);
        st.acc3[a * k + b].release();
      }
      out[a * k + b] = rescale(st.acc[a * k + b]);
      st.acc[a * k + b] = HeCt();
    }
  for (int a = 0; a < k; a++)
    for (int b = a + 1; b < k; b++) out[a * k + b] = lintrans(out[b * k + a], LT_TRANSPOSE, n, st.n1g, 1.0);
  if (k > 1) {
    int fl = out[1].level;
    for (int a = 0; a < k; a++)
      for (int b = 0; b <= a; b++) out[a * k + b] = drop(out[a * k + b], fl);
  }
  st.row_blocks = 0;
  st.set.assign(k * k, false);
  return out;
}

std::vector<HeCt> HeCtxImpl::covariance(const std::vector<const HeCt*>& x, int rb, int k, int n, u64 n_samples,
                                        int n1z, int n1t, int n1g, int npz, int npt, bool lazy,
                                        bool fused_rs) {
  if ((int)x.size() != rb * k) fail(HE_EINVAL, "block count mismatch");
  CovState st = cov_begin(k, n, n_samples, n1z, n1t, n1g, npz, npt, lazy, fused_rs);
  cov_add(st, x, rb);
  return cov_end(st);
}
