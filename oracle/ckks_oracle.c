/*
 * Plain CPU oracle for the RNS-CKKS homomorphic matrix product of
 * "Improved Privacy-Preserving PCA Using Optimized Homomorphic Matrix
 * Multiplication" (arXiv 2305.17341).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file; only the test-suite, the smoke check and the CPU-baseline
 * leg of the benchmark use it.  It shares no code, header, table or constant
 * generator with the HIP library: every definition here is written out again
 * from the paper (and from the published definitions it relies on).
 *
 * Style: slow and literal.  Every modular product is (a*b) % q on 128-bit
 * integers, every transform is the textbook loop, nothing is fused.  OpenMP
 * pragmas only split independent limbs / coefficients across threads and do
 * not change any result.
 *
 * Conventions (paper Appendix A, "full-RNS CKKS"; notation section):
 *   - a ciphertext at level l lives in R_{Q_l}^2 with Q_l = q_0 ... q_l and is
 *     stored limb-major: u64[2][l+1][N], every limb in the NTT (evaluation)
 *     domain, residues in [0, q).
 *   - the special modulus P = p_0 ... p_{alpha-1}; an element of R_{Q_l P} is
 *     stored as l+1 Q limbs followed by alpha P limbs.
 *   - [x]_q is the centred residue in (-q/2, q/2]; "x mod q" is in [0, q).
 */
#include <math.h>
#include <omp.h>
#include <quadmath.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

typedef uint64_t u64;
typedef int64_t i64;
typedef unsigned __int128 u128;

#define MAXMOD 64

/* ------------------------------------------------------------------------ */
/* Scalar modular arithmetic                                                 */
/* ------------------------------------------------------------------------ */
static u64 mulmod(u64 a, u64 b, u64 q) { return (u64)(((u128)a * b) % q); }
static u64 addmod(u64 a, u64 b, u64 q) { return (u64)(((u128)a + b) % q); }
static u64 submod(u64 a, u64 b, u64 q) { return (u64)(((u128)a + q - b) % q); }
static u64 powmod(u64 b, u64 e, u64 q) {
  u64 r = 1 % q;
  b %= q;
  while (e) {
    if (e & 1) r = mulmod(r, b, q);
    b = mulmod(b, b, q);
    e >>= 1;
  }
  return r;
}
/* q prime: Fermat inverse */
static u64 invmod(u64 a, u64 q) { return powmod(a % q, q - 2, q); }
/* reduce a signed integer into [0, q) */
static u64 smod(i64 v, u64 q) {
  i64 r = v % (i64)q;
  return (u64)(r < 0 ? r + (i64)q : r);
}

/* ------------------------------------------------------------------------ */
/* Parameter generation (Appendix A, Setparams): primes q_i, p_i = 1 mod 2N  */
/* ------------------------------------------------------------------------ */
/* Deterministic Miller-Rabin for 64-bit integers (the first 12 prime bases
 * are a proven witness set below 3.3e24). */
static int is_prime_u64(u64 n) {
  static const u64 bases[12] = {2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37};
  if (n < 2) return 0;
  for (int i = 0; i < 12; i++) {
    if (n == bases[i]) return 1;
    if (n % bases[i] == 0) return 0;
  }
  u64 d = n - 1;
  int s = 0;
  while ((d & 1) == 0) { d >>= 1; s++; }
  for (int i = 0; i < 12; i++) {
    u64 x = powmod(bases[i], d, n);
    if (x == 1 || x == n - 1) continue;
    int comp = 1;
    for (int r = 1; r < s; r++) {
      x = mulmod(x, x, n);
      if (x == n - 1) { comp = 0; break; }
    }
    if (comp) return 0;
  }
  return 1;
}

/* Reading of Setparams: for each bit size b the candidates are 1 + t*2N just
 * below 2^b, scanned downward; Q takes them first (in the order the chain
 * lists them), then P takes the next unused ones of its bit sizes. */
static int gen_primes(int logN, const int *qbits, int nq, const int *pbits,
                      int np, u64 *out) {
  u64 twoN = 2ull << logN;
  u64 cursor[65];
  for (int b = 0; b <= 64; b++) cursor[b] = 0;
  int total = nq + np;
  for (int k = 0; k < total; k++) {
    int b = k < nq ? qbits[k] : pbits[k - nq];
    if (b < 20 || b > 61) return -1;
    if (cursor[b] == 0) cursor[b] = ((1ull << b) - 2) / twoN; /* q <= 2^b - 1 */
    for (;;) {
      u64 t = cursor[b];
      if (t == 0) return -1;
      cursor[b] = t - 1;
      u64 q = t * twoN + 1;
      if (q < (1ull << (b - 1))) return -1;
      if (is_prime_u64(q)) { out[k] = q; break; }
    }
  }
  return total;
}

/* Primitive 2N-th root: psi = x^((q-1)/2N) for the smallest x >= 2 with
 * psi^N = -1 (mod q). */
static u64 find_psi(u64 q, int logN) {
  u64 N = 1ull << logN;
  for (u64 x = 2;; x++) {
    u64 psi = powmod(x, (q - 1) / (2 * N), q);
    if (powmod(psi, N, q) == q - 1) return psi;
  }
}

static u64 bitrev(u64 x, int bits) {
  u64 r = 0;
  for (int i = 0; i < bits; i++) r |= ((x >> i) & 1ull) << (bits - 1 - i);
  return r;
}

/* ------------------------------------------------------------------------ */
/* Counter-based randomness: Philox4x64-10 (Salmon, Moraes, Dror, Shaw,      */
/* "Parallel random numbers: as easy as 1, 2, 3", SC'11).                    */
/* ------------------------------------------------------------------------ */
void oc_philox4x64(const u64 ctr_in[4], const u64 key_in[2], u64 out[4]) {
  const u64 M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
  const u64 W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
  u64 c[4] = {ctr_in[0], ctr_in[1], ctr_in[2], ctr_in[3]};
  u64 k0 = key_in[0], k1 = key_in[1];
  for (int r = 0; r < 10; r++) {
    if (r > 0) { k0 += W0; k1 += W1; }
    u128 p0 = (u128)M0 * c[0];
    u128 p1 = (u128)M1 * c[2];
    u64 hi0 = (u64)(p0 >> 64), lo0 = (u64)p0;
    u64 hi1 = (u64)(p1 >> 64), lo1 = (u64)p1;
    u64 n0 = hi1 ^ c[1] ^ k0, n1 = lo1, n2 = hi0 ^ c[3] ^ k1, n3 = lo0;
    c[0] = n0; c[1] = n1; c[2] = n2; c[3] = n3;
  }
  out[0] = c[0]; out[1] = c[1]; out[2] = c[2]; out[3] = c[3];
}

/* Randomness streams: key = (ctx seed, tag), counter = (coefficient index,
 * limb, object, sub-object).  Tags name what is drawn. */
enum {
  TAG_SK = 1, TAG_PK_A = 2, TAG_PK_E = 3, TAG_SWK_A = 4, TAG_SWK_E = 5,
  TAG_ENC_V = 6, TAG_ENC_E0 = 7, TAG_ENC_E1 = 8
};

static void draw(u64 seed, u64 tag, u64 c0, u64 c1, u64 c2, u64 c3, u64 out[4]) {
  u64 ctr[4] = {c0, c1, c2, c3};
  u64 key[2] = {seed, tag};
  oc_philox4x64(ctr, key, out);
}

/* Truncated discrete Gaussian (Appendix A, chi_e), width sigma, support
 * |x| <= 19, sampled by inversion of its cumulative table. */
#define CDT_HALF 19
#define CDT_LEN (2 * CDT_HALF)
void oc_cdt_table(double sigma, u64 *table) {
  double rho[2 * CDT_HALF + 1];
  double z = 0.0;
  for (int x = -CDT_HALF; x <= CDT_HALF; x++) {
    rho[x + CDT_HALF] = exp(-((double)x * (double)x) / (2.0 * sigma * sigma));
  }
  for (int k = 0; k < 2 * CDT_HALF + 1; k++) z += rho[k];
  double cum = 0.0;
  for (int k = 0; k < CDT_LEN; k++) {
    cum += rho[k];
    table[k] = (u64)(cum / z * 18446744073709551616.0);
  }
}
static int cdt_sample(const u64 *table, u64 w) {
  int x = -CDT_HALF;
  for (int k = 0; k < CDT_LEN; k++)
    if (w >= table[k]) x++;
  return x;
}
static int ternary_from(u64 w) { return (int)(w % 3) - 1; }
static u64 uniform_from(u64 w0, u64 w1, u64 q) {
  u128 x = ((u128)w0 << 64) | w1;
  return (u64)(x % q);
}

/* ------------------------------------------------------------------------ */
/* Context                                                                   */
/* ------------------------------------------------------------------------ */
typedef struct {
  u64 galois; /* 0 = relinearisation key */
  u64 *data;  /* [beta][2][L+1+alpha][N] */
} oc_key;

typedef struct oc_ctx {
  int logN;
  u64 N;
  int L;     /* top level: Q has L+1 primes */
  int alpha; /* number of special primes */
  int beta;  /* digits at the top level = ceil((L+1)/alpha) */
  int nmods;
  u64 mods[MAXMOD]; /* q_0..q_L, p_0..p_{alpha-1} */
  u64 psi[MAXMOD];
  u64 *psi_rev[MAXMOD];
  u64 *psi_inv_rev[MAXMOD];
  u64 ninv[MAXMOD];
  double delta; /* default scale 2^log2_scale */
  double sigma;
  u64 seed;
  u64 cdt[CDT_LEN];
  int8_t *s;  /* secret key coefficients */
  u64 *s_ntt; /* [nmods][N] */
  u64 *pk;    /* [2][L+1][N] */
  int nkeys;
  oc_key keys[512];
  int have_sk;
} oc_ctx;

typedef struct oc_ct {
  int level;
  int nlimbs; /* l+1 (or l+1+alpha for QP elements) */
  int qp;     /* 1 if the element lives in R_{Q_l P} */
  double scale;
  u64 *d; /* [2][nlimbs][N] */
} oc_ct;

static u64 *alloc_u64(size_t n) {
  u64 *p = (u64 *)calloc(n, sizeof(u64));
  if (!p) { fprintf(stderr, "oracle: out of memory (%zu words)\n", n); abort(); }
  return p;
}

oc_ctx *oc_create(int logN, const int *qbits, int nq, const int *pbits, int np,
                  double log2_scale, double sigma, u64 seed) {
  if (logN < 2 || logN > 17 || nq < 1 || np < 1 || nq + np > MAXMOD) return NULL;
  oc_ctx *c = (oc_ctx *)calloc(1, sizeof(oc_ctx));
  c->logN = logN;
  c->N = 1ull << logN;
  c->L = nq - 1;
  c->alpha = np;
  c->beta = (nq + np - 1) / np;
  c->nmods = nq + np;
  if (gen_primes(logN, qbits, nq, pbits, np, c->mods) != nq + np) { free(c); return NULL; }
  for (int m = 0; m < c->nmods; m++) {
    u64 q = c->mods[m];
    c->psi[m] = find_psi(q, logN);
    u64 psinv = invmod(c->psi[m], q);
    c->psi_rev[m] = alloc_u64(c->N);
    c->psi_inv_rev[m] = alloc_u64(c->N);
    /* successive powers psi^k, psi^-k, then placed at bit-reversed k */
    u64 pw = 1, pwi = 1;
    for (u64 k = 0; k < c->N; k++) {
      u64 e = bitrev(k, logN);
      c->psi_rev[m][e] = pw;
      c->psi_inv_rev[m][e] = pwi;
      pw = mulmod(pw, c->psi[m], q);
      pwi = mulmod(pwi, psinv, q);
    }
    c->ninv[m] = invmod(c->N % q, q);
  }
  c->delta = ldexp(1.0, 0) * pow(2.0, log2_scale);
  c->sigma = sigma;
  c->seed = seed;
  oc_cdt_table(sigma, c->cdt);
  return c;
}

void oc_destroy(oc_ctx *c) {
  if (!c) return;
  for (int m = 0; m < c->nmods; m++) { free(c->psi_rev[m]); free(c->psi_inv_rev[m]); }
  free(c->s); free(c->s_ntt); free(c->pk);
  for (int k = 0; k < c->nkeys; k++) free(c->keys[k].data);
  free(c);
}

int oc_nmods(const oc_ctx *c) { return c->nmods; }
void oc_moduli(const oc_ctx *c, u64 *out) { memcpy(out, c->mods, sizeof(u64) * c->nmods); }
u64 oc_psi(const oc_ctx *c, int m) { return c->psi[m]; }
int oc_L(const oc_ctx *c) { return c->L; }
int oc_alpha(const oc_ctx *c) { return c->alpha; }
void oc_cdt(const oc_ctx *c, u64 *out) { memcpy(out, c->cdt, sizeof(c->cdt)); }

/* index of a Q-or-P limb position within a QP element of level l */
static int qp_mod_index(const oc_ctx *c, int level, int pos) {
  return pos <= level ? pos : c->L + 1 + (pos - level - 1);
}

/* ------------------------------------------------------------------------ */
/* Negacyclic NTT (RNS + NTT representation, section 3.2 / Appendix A).       */
/* Layout: output index i holds a(psi^(2*brv(i)+1)).                         */
/* ------------------------------------------------------------------------ */
void oc_ntt(const oc_ctx *c, int m, u64 *a) {
  u64 q = c->mods[m], N = c->N;
  u64 t = N;
  for (u64 mm = 1; mm < N; mm <<= 1) {
    t >>= 1;
    for (u64 i = 0; i < mm; i++) {
      u64 w = c->psi_rev[m][mm + i];
      u64 j1 = 2 * i * t;
      for (u64 j = j1; j < j1 + t; j++) {
        u64 u = a[j], v = mulmod(a[j + t], w, q);
        a[j] = addmod(u, v, q);
        a[j + t] = submod(u, v, q);
      }
    }
  }
}

void oc_intt(const oc_ctx *c, int m, u64 *a) {
  u64 q = c->mods[m], N = c->N;
  u64 t = 1;
  for (u64 mm = N; mm > 1; mm >>= 1) {
    u64 h = mm >> 1, j1 = 0;
    for (u64 i = 0; i < h; i++) {
      u64 w = c->psi_inv_rev[m][h + i];
      for (u64 j = j1; j < j1 + t; j++) {
        u64 u = a[j], v = a[j + t];
        a[j] = addmod(u, v, q);
        a[j + t] = mulmod(submod(u, v, q), w, q);
      }
      j1 += 2 * t;
    }
    t <<= 1;
  }
  for (u64 j = 0; j < N; j++) a[j] = mulmod(a[j], c->ninv[m], q);
}

/* The definition itself (for pins at small N): out[i] = a(psi^(2 brv(i)+1)). */
void oc_ntt_direct(const oc_ctx *c, int m, const u64 *a, u64 *out) {
  u64 q = c->mods[m], N = c->N;
  for (u64 i = 0; i < N; i++) {
    u64 x = powmod(c->psi[m], 2 * bitrev(i, c->logN) + 1, q);
    u64 acc = 0, xp = 1;
    for (u64 k = 0; k < N; k++) {
      acc = addmod(acc, mulmod(a[k], xp, q), q);
      xp = mulmod(xp, x, q);
    }
    out[i] = acc;
  }
}

static void ntt_limbs(const oc_ctx *c, u64 *d, const int *modidx, int nl) {
#pragma omp parallel for schedule(dynamic)
  for (int k = 0; k < nl; k++) oc_ntt(c, modidx[k], d + (size_t)k * c->N);
}
static void intt_limbs(const oc_ctx *c, u64 *d, const int *modidx, int nl) {
#pragma omp parallel for schedule(dynamic)
  for (int k = 0; k < nl; k++) oc_intt(c, modidx[k], d + (size_t)k * c->N);
}

/* ------------------------------------------------------------------------ */
/* Galois automorphism X -> X^g (rotation, Appendix A "Rot").                */
/* ------------------------------------------------------------------------ */
/* NTT domain: slot i holds a(psi^(2 brv(i)+1)); a(X^g) evaluated there is a at
 * psi^(g (2 brv(i)+1)), which sits at index brv((g(2brv(i)+1) mod 2N - 1)/2). */
void oc_automorph_ntt(const oc_ctx *c, u64 g, const u64 *in, u64 *out) {
  u64 N = c->N, twoN = 2 * N;
  for (u64 i = 0; i < N; i++) {
    u64 e = (g * (2 * bitrev(i, c->logN) + 1)) % twoN;
    out[i] = in[bitrev((e - 1) / 2, c->logN)];
  }
}
/* coefficient domain: a_k X^k -> a_k X^(gk mod 2N) with X^N = -1 */
void oc_automorph_coef(const oc_ctx *c, int m, u64 g, const u64 *in, u64 *out) {
  u64 N = c->N, twoN = 2 * N, q = c->mods[m];
  for (u64 k = 0; k < N; k++) {
    u64 e = (g * k) % twoN;
    if (e < N) out[e] = in[k];
    else out[e - N] = in[k] == 0 ? 0 : q - in[k];
  }
}

/* Galois element of a left rotation by k slots: 5^(k mod N/2) mod 2N. */
u64 oc_galois_of_step(const oc_ctx *c, i64 k) {
  i64 slots = (i64)(c->N / 2);
  i64 r = ((k % slots) + slots) % slots;
  u64 g = 1, twoN = 2 * c->N;
  for (i64 i = 0; i < r; i++) g = (g * 5) % twoN;
  return g;
}

/* ------------------------------------------------------------------------ */
/* Encoding (Appendix A "Encode"): canonical embedding at the slots          */
/* zeta^(5^j), zeta = exp(i pi / N), with real messages.                     */
/*   v_i = (2 Delta / N) sum_{j < N/2} z_j cos(pi (5^j i mod 2N) / N)          */
/*   m_i = floor(v_i + 1/2 + 2^-30)                                          */
/* (round to nearest; values within 2^-30 below a half-integer go up, so     */
/* exact ties are decided the same way by any sufficiently precise encoder).  */
/* A message shorter than N/2 is replicated with its own period.             */
/* ------------------------------------------------------------------------ */
static const __float128 ENC_EPS = 9.31322574615478515625e-10Q; /* 2^-30 */

/* Definition written out: O(N^2), quad precision.  For pins at small N. */
int oc_encode_direct(const oc_ctx *c, const double *z, int nz, double delta, i64 *out) {
  u64 N = c->N, twoN = 2 * N, S = N / 2;
  if (nz <= 0 || S % (u64)nz) return -1;
  __float128 *cosv = (__float128 *)malloc(sizeof(__float128) * twoN);
  for (u64 e = 0; e < twoN; e++) cosv[e] = cosq(M_PIq * (__float128)e / (__float128)N);
  u64 *pw = alloc_u64(S);
  u64 g = 1;
  for (u64 j = 0; j < S; j++) { pw[j] = g; g = (g * 5) % twoN; }
#pragma omp parallel for schedule(static)
  for (u64 i = 0; i < N; i++) {
    __float128 acc = 0;
    for (u64 j = 0; j < S; j++) acc += (__float128)z[j % nz] * cosv[(pw[j] * i) % twoN];
    __float128 v = acc * 2 * (__float128)delta / (__float128)N;
    out[i] = (i64)floorq(v + 0.5Q + ENC_EPS);
  }
  free(cosv); free(pw);
  return 0;
}

/* Same quantity through a length-N complex FFT in quad precision:
 * with u[t] = z_j for odd 2t+1 = +-5^j mod 2N,
 *   v_i = (Delta/N) Re( zeta^(-i) sum_t u[t] w^(-t i) ),  w = exp(2 pi i/N). */
static void fft_q(__complex128 *x, u64 N, int logN, int inverse_sign) {
  for (u64 i = 0; i < N; i++) {
    u64 j = bitrev(i, logN);
    if (j > i) { __complex128 t = x[i]; x[i] = x[j]; x[j] = t; }
  }
  __complex128 *tw = (__complex128 *)malloc(sizeof(__complex128) * (N / 2));
  for (u64 k = 0; k < N / 2; k++) {
    __float128 ang = 2 * M_PIq * (__float128)k / (__float128)N;
    __real__ tw[k] = cosq(ang);
    __imag__ tw[k] = inverse_sign * sinq(ang);
  }
  for (u64 len = 2; len <= N; len <<= 1) {
    u64 stride = N / len;
    for (u64 s = 0; s < N; s += len) {
      for (u64 k = 0; k < len / 2; k++) {
        __complex128 w = tw[k * stride];
        __complex128 a = x[s + k], b = x[s + k + len / 2] * w;
        x[s + k] = a + b;
        x[s + k + len / 2] = a - b;
      }
    }
  }
  free(tw);
}

int oc_encode(const oc_ctx *c, const double *z, int nz, double delta, i64 *out) {
  u64 N = c->N, twoN = 2 * N, S = N / 2;
  if (nz <= 0 || S % (u64)nz) return -1;
  __complex128 *u = (__complex128 *)calloc(N, sizeof(__complex128));
  u64 g = 1;
  for (u64 j = 0; j < S; j++) {
    __float128 zj = (__float128)z[j % nz];
    __real__ u[(g - 1) / 2] = zj;
    __real__ u[(twoN - g - 1) / 2] = zj;
    g = (g * 5) % twoN;
  }
  fft_q(u, N, c->logN, -1); /* sum_t u[t] w^(-t i) */
  for (u64 i = 0; i < N; i++) {
    __float128 ang = M_PIq * (__float128)i / (__float128)N;
    __float128 re = crealq(u[i]) * cosq(ang) + cimagq(u[i]) * sinq(ang);
    __float128 v = re * (__float128)delta / (__float128)N;
    out[i] = (i64)floorq(v + 0.5Q + ENC_EPS);
  }
  free(u);
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Ciphertext containers and elementary operations (Appendix A)              */
/* ------------------------------------------------------------------------ */
static oc_ct *ct_new(const oc_ctx *c, int level, int qp, double scale) {
  oc_ct *r = (oc_ct *)calloc(1, sizeof(oc_ct));
  r->level = level;
  r->qp = qp;
  r->nlimbs = level + 1 + (qp ? c->alpha : 0);
  r->scale = scale;
  r->d = alloc_u64((size_t)2 * r->nlimbs * c->N);
  return r;
}
void oc_ct_free(oc_ct *x) { if (x) { free(x->d); free(x); } }
void oc_free(void *p) { free(p); }
int oc_ct_level(const oc_ct *x) { return x->level; }
double oc_ct_scale(const oc_ct *x) { return x->scale; }
int oc_ct_nlimbs(const oc_ct *x) { return x->nlimbs; }
u64 *oc_ct_data(oc_ct *x) { return x->d; }
static u64 *poly(const oc_ctx *c, const oc_ct *x, int p, int limb) {
  return x->d + ((size_t)p * x->nlimbs + limb) * c->N;
}
static int limb_mod(const oc_ctx *c, const oc_ct *x, int limb) {
  return x->qp ? qp_mod_index(c, x->level, limb) : limb;
}

oc_ct *oc_ct_import(const oc_ctx *c, const u64 *data, int level, int qp, double scale) {
  oc_ct *r = ct_new(c, level, qp, scale);
  memcpy(r->d, data, sizeof(u64) * 2 * r->nlimbs * c->N);
  return r;
}
oc_ct *oc_ct_copy(const oc_ctx *c, const oc_ct *x) {
  return oc_ct_import(c, x->d, x->level, x->qp, x->scale);
}

/* integer polynomial -> NTT-domain residues for the given modulus indices */
static void poly_from_int(const oc_ctx *c, const i64 *m, const int *modidx, int nl, u64 *out) {
  for (int k = 0; k < nl; k++) {
    u64 q = c->mods[modidx[k]];
    for (u64 i = 0; i < c->N; i++) out[(size_t)k * c->N + i] = smod(m[i], q);
  }
  ntt_limbs(c, out, modidx, nl);
}

/* ------------------------------------------------------------------------ */
/* Key generation (Appendix A: SecKeyGen, PubKeyGen, SwitchKeyGen)           */
/* ------------------------------------------------------------------------ */
static void gauss_poly(const oc_ctx *c, u64 tag, u64 c1, u64 c2, u64 c3, i64 *e) {
  for (u64 i = 0; i < c->N; i++) {
    u64 w[4];
    draw(c->seed, tag, i, c1, c2, c3, w);
    e[i] = cdt_sample(c->cdt, w[0]);
  }
}

void oc_keygen_secret(oc_ctx *c) {
  u64 N = c->N;
  c->s = (int8_t *)malloc(N);
  for (u64 i = 0; i < N; i++) {
    u64 w[4];
    draw(c->seed, TAG_SK, i, 0, 0, 0, w);
    c->s[i] = (int8_t)ternary_from(w[0]);
  }
  c->s_ntt = alloc_u64((size_t)c->nmods * N);
  int idx[MAXMOD];
  i64 *si = (i64 *)malloc(sizeof(i64) * N);
  for (u64 i = 0; i < N; i++) si[i] = c->s[i];
  for (int m = 0; m < c->nmods; m++) idx[m] = m;
  poly_from_int(c, si, idx, c->nmods, c->s_ntt);
  free(si);
  /* public key (-a s + e, a) over Q_L */
  c->pk = alloc_u64((size_t)2 * (c->L + 1) * N);
  i64 *e = (i64 *)malloc(sizeof(i64) * N);
  gauss_poly(c, TAG_PK_E, 0, 0, 0, e);
  u64 *en = alloc_u64((size_t)(c->L + 1) * N);
  poly_from_int(c, e, idx, c->L + 1, en);
  for (int m = 0; m <= c->L; m++) {
    u64 q = c->mods[m];
    for (u64 i = 0; i < N; i++) {
      u64 w[4];
      draw(c->seed, TAG_PK_A, i, (u64)m, 0, 0, w);
      u64 a = uniform_from(w[0], w[1], q);
      u64 as = mulmod(a, c->s_ntt[(size_t)m * N + i], q);
      c->pk[(size_t)m * N + i] = addmod(submod(0, as, q), en[(size_t)m * N + i], q);
      c->pk[(size_t)(c->L + 1 + m) * N + i] = a;
    }
  }
  free(e); free(en);
  c->have_sk = 1;
}

/* Switching key from s' (given in NTT form over all Q and P moduli) to s.
 * Digit j covers q_{j alpha} .. q_{j alpha + alpha - 1}.  Component j:
 *   b_j = -a_j s + e_j + P [q_t in D_j] s'   (mod every Q and P prime t)
 *   a_j uniform, drawn directly in the NTT domain.
 * kid names the key in the randomness stream (0 = relinearisation,
 * otherwise the Galois element). */
static void swk_gen(oc_ctx *c, const u64 *sp_ntt, u64 kid, u64 *out) {
  u64 N = c->N;
  int nm = c->nmods;
  int idx[MAXMOD];
  for (int m = 0; m < nm; m++) idx[m] = m;
  i64 *e = (i64 *)malloc(sizeof(i64) * N);
  u64 *en = alloc_u64((size_t)nm * N);
  for (int j = 0; j < c->beta; j++) {
    gauss_poly(c, TAG_SWK_E, 0, (u64)j, kid, e);
    poly_from_int(c, e, idx, nm, en);
    u64 *bj = out + ((size_t)j * 2 + 0) * nm * N;
    u64 *aj = out + ((size_t)j * 2 + 1) * nm * N;
#pragma omp parallel for schedule(static)
    for (int m = 0; m < nm; m++) {
      u64 q = c->mods[m];
      u64 pmod = 1;
      for (int k = 0; k < c->alpha; k++) pmod = mulmod(pmod, c->mods[c->L + 1 + k] % q, q);
      int in_digit = (m <= c->L) && (m / c->alpha == j);
      for (u64 i = 0; i < N; i++) {
        u64 w[4];
        draw(c->seed, TAG_SWK_A, i, (u64)m, (u64)j, kid, w);
        u64 a = uniform_from(w[0], w[1], q);
        u64 v = submod(en[(size_t)m * N + i], mulmod(a, c->s_ntt[(size_t)m * N + i], q), q);
        if (in_digit) v = addmod(v, mulmod(pmod, sp_ntt[(size_t)m * N + i], q), q);
        bj[(size_t)m * N + i] = v;
        aj[(size_t)m * N + i] = a;
      }
    }
  }
  free(e); free(en);
}

static oc_key *find_key(const oc_ctx *c, u64 galois) {
  for (int k = 0; k < c->nkeys; k++)
    if (c->keys[k].galois == galois) return (oc_key *)&c->keys[k];
  return NULL;
}

/* relinearisation key (s' = s^2) */
int oc_keygen_relin(oc_ctx *c) {
  if (!c->have_sk) return -1;
  if (find_key(c, 0)) return 0;
  u64 N = c->N;
  u64 *s2 = alloc_u64((size_t)c->nmods * N);
  for (int m = 0; m < c->nmods; m++)
    for (u64 i = 0; i < N; i++) {
      u64 v = c->s_ntt[(size_t)m * N + i];
      s2[(size_t)m * N + i] = mulmod(v, v, c->mods[m]);
    }
  oc_key *k = &c->keys[c->nkeys++];
  k->galois = 0;
  k->data = alloc_u64((size_t)c->beta * 2 * c->nmods * N);
  swk_gen(c, s2, 0, k->data);
  free(s2);
  return 0;
}

/* rotation key for a left rotation by `step` slots (s' = s(X^g)) */
int oc_keygen_rot(oc_ctx *c, i64 step) {
  if (!c->have_sk) return -1;
  u64 g = oc_galois_of_step(c, step);
  if (g == 1 || find_key(c, g)) return 0;
  if (c->nkeys >= 512) return -2;
  u64 N = c->N;
  u64 *sg = alloc_u64((size_t)c->nmods * N);
  for (int m = 0; m < c->nmods; m++)
    oc_automorph_ntt(c, g, c->s_ntt + (size_t)m * N, sg + (size_t)m * N);
  oc_key *k = &c->keys[c->nkeys++];
  k->galois = g;
  k->data = alloc_u64((size_t)c->beta * 2 * c->nmods * N);
  swk_gen(c, sg, g, k->data);
  free(sg);
  return 0;
}

/* secret key coefficients (client side; for tests) */
void oc_secret(const oc_ctx *c, int8_t *out) { memcpy(out, c->s, c->N); }

/* ------------------------------------------------------------------------ */
/* Encryption / decryption (Appendix A: Enc, Dec)                            */
/* ------------------------------------------------------------------------ */
/* ct = (v pk0 + m + e0, v pk1 + e1) over Q_level, v ternary, e0,e1 Gaussian. */
oc_ct *oc_encrypt_poly(oc_ctx *c, const i64 *m, int level, double scale, u64 nonce) {
  if (!c->have_sk || level < 0 || level > c->L) return NULL;
  u64 N = c->N;
  int nl = level + 1;
  int idx[MAXMOD];
  for (int k = 0; k < nl; k++) idx[k] = k;
  i64 *v = (i64 *)malloc(sizeof(i64) * N), *e0 = (i64 *)malloc(sizeof(i64) * N),
      *e1 = (i64 *)malloc(sizeof(i64) * N);
  for (u64 i = 0; i < N; i++) {
    u64 w[4];
    draw(c->seed, TAG_ENC_V, i, 0, nonce, 0, w);
    v[i] = ternary_from(w[0]);
  }
  gauss_poly(c, TAG_ENC_E0, 0, nonce, 0, e0);
  gauss_poly(c, TAG_ENC_E1, 0, nonce, 0, e1);
  for (u64 i = 0; i < N; i++) e0[i] += m[i];
  u64 *vn = alloc_u64((size_t)nl * N), *m0 = alloc_u64((size_t)nl * N),
      *m1 = alloc_u64((size_t)nl * N);
  poly_from_int(c, v, idx, nl, vn);
  poly_from_int(c, e0, idx, nl, m0);
  poly_from_int(c, e1, idx, nl, m1);
  oc_ct *r = ct_new(c, level, 0, scale);
  for (int k = 0; k < nl; k++) {
    u64 q = c->mods[k];
    for (u64 i = 0; i < N; i++) {
      size_t o = (size_t)k * N + i;
      poly(c, r, 0, k)[i] = addmod(mulmod(vn[o], c->pk[o], q), m0[o], q);
      poly(c, r, 1, k)[i] =
          addmod(mulmod(vn[o], c->pk[(size_t)(c->L + 1 + k) * N + i], q), m1[o], q);
    }
  }
  free(v); free(e0); free(e1); free(vn); free(m0); free(m1);
  return r;
}

oc_ct *oc_encrypt(oc_ctx *c, const double *z, int nz, int level, u64 nonce) {
  i64 *m = (i64 *)malloc(sizeof(i64) * c->N);
  if (oc_encode(c, z, nz, c->delta, m)) { free(m); return NULL; }
  oc_ct *r = oc_encrypt_poly(c, m, level, c->delta, nonce);
  free(m);
  return r;
}

/* Dec: c0 + c1 s, returned as coefficient-domain residues u64[l+1][N]. */
int oc_decrypt_residues(const oc_ctx *c, const oc_ct *x, u64 *out) {
  if (!c->have_sk || x->qp) return -1;
  u64 N = c->N;
  int nl = x->level + 1;
  int idx[MAXMOD];
  for (int k = 0; k < nl; k++) {
    idx[k] = k;
    u64 q = c->mods[k];
    for (u64 i = 0; i < N; i++)
      out[(size_t)k * N + i] =
          addmod(poly(c, x, 0, k)[i], mulmod(poly(c, x, 1, k)[i], c->s_ntt[(size_t)k * N + i], q), q);
  }
  intt_limbs(c, out, idx, nl);
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Add / Sub / PMult / Tensor / Rescale (Appendix A, addition and            */
/* multiplication modules)                                                   */
/* ------------------------------------------------------------------------ */
static int same_shape(const oc_ct *a, const oc_ct *b) {
  return a->level == b->level && a->qp == b->qp;
}
oc_ct *oc_add(const oc_ctx *c, const oc_ct *a, const oc_ct *b) {
  if (!same_shape(a, b)) return NULL;
  oc_ct *r = ct_new(c, a->level, a->qp, a->scale);
  for (int p = 0; p < 2; p++)
    for (int k = 0; k < a->nlimbs; k++) {
      u64 q = c->mods[limb_mod(c, a, k)];
      for (u64 i = 0; i < c->N; i++) poly(c, r, p, k)[i] = addmod(poly(c, a, p, k)[i], poly(c, b, p, k)[i], q);
    }
  return r;
}
oc_ct *oc_sub(const oc_ctx *c, const oc_ct *a, const oc_ct *b) {
  if (!same_shape(a, b)) return NULL;
  oc_ct *r = ct_new(c, a->level, a->qp, a->scale);
  for (int p = 0; p < 2; p++)
    for (int k = 0; k < a->nlimbs; k++) {
      u64 q = c->mods[limb_mod(c, a, k)];
      for (u64 i = 0; i < c->N; i++) poly(c, r, p, k)[i] = submod(poly(c, a, p, k)[i], poly(c, b, p, k)[i], q);
    }
  return r;
}
static void add_into(const oc_ctx *c, oc_ct *acc, const oc_ct *b) {
  for (int p = 0; p < 2; p++)
    for (int k = 0; k < acc->nlimbs; k++) {
      u64 q = c->mods[limb_mod(c, acc, k)];
      for (u64 i = 0; i < c->N; i++) poly(c, acc, p, k)[i] = addmod(poly(c, acc, p, k)[i], poly(c, b, p, k)[i], q);
    }
}

/* PMult: (c0 m, c1 m), scale multiplies.  m given as integer coefficients. */
oc_ct *oc_pmult(const oc_ctx *c, const oc_ct *a, const i64 *m, double pt_scale) {
  int nl = a->nlimbs, idx[MAXMOD];
  for (int k = 0; k < nl; k++) idx[k] = limb_mod(c, a, k);
  u64 *mn = alloc_u64((size_t)nl * c->N);
  poly_from_int(c, m, idx, nl, mn);
  oc_ct *r = ct_new(c, a->level, a->qp, a->scale * pt_scale);
  for (int p = 0; p < 2; p++)
    for (int k = 0; k < nl; k++) {
      u64 q = c->mods[idx[k]];
      for (u64 i = 0; i < c->N; i++)
        poly(c, r, p, k)[i] = mulmod(poly(c, a, p, k)[i], mn[(size_t)k * c->N + i], q);
    }
  free(mn);
  return r;
}

/* PAdd: (c0 + m, c1) for a plaintext m given as integer coefficients at the
 * ciphertext's scale (Appendix A, addition module). */
oc_ct *oc_padd(const oc_ctx *c, const oc_ct *a, const i64 *m) {
  int nl = a->nlimbs, idx[MAXMOD];
  for (int k = 0; k < nl; k++) idx[k] = limb_mod(c, a, k);
  u64 *mn = alloc_u64((size_t)nl * c->N);
  poly_from_int(c, m, idx, nl, mn);
  oc_ct *r = oc_ct_copy(c, a);
  for (int k = 0; k < nl; k++) {
    u64 q = c->mods[idx[k]];
    for (u64 i = 0; i < c->N; i++) poly(c, r, 0, k)[i] = addmod(poly(c, a, 0, k)[i], mn[(size_t)k * c->N + i], q);
  }
  free(mn);
  return r;
}

/* multiplication by a small integer constant (no level consumed) */
oc_ct *oc_mul_int(const oc_ctx *c, const oc_ct *a, i64 k) {
  oc_ct *r = ct_new(c, a->level, a->qp, a->scale);
  for (int p = 0; p < 2; p++)
    for (int l = 0; l < a->nlimbs; l++) {
      u64 q = c->mods[limb_mod(c, a, l)], kk = smod(k, q);
      for (u64 i = 0; i < c->N; i++) poly(c, r, p, l)[i] = mulmod(poly(c, a, p, l)[i], kk, q);
    }
  return r;
}

/* Tensor (first half of Mult): (a0 b0, a0 b1 + a1 b0, a1 b1); the three
 * components are returned in out[3][l+1][N]. */
int oc_tensor(const oc_ctx *c, const oc_ct *a, const oc_ct *b, u64 *out) {
  if (!same_shape(a, b) || a->qp) return -1;
  u64 N = c->N;
  int nl = a->nlimbs;
  for (int k = 0; k < nl; k++) {
    u64 q = c->mods[k];
    for (u64 i = 0; i < N; i++) {
      u64 a0 = poly(c, a, 0, k)[i], a1 = poly(c, a, 1, k)[i];
      u64 b0 = poly(c, b, 0, k)[i], b1 = poly(c, b, 1, k)[i];
      out[((size_t)0 * nl + k) * N + i] = mulmod(a0, b0, q);
      out[((size_t)1 * nl + k) * N + i] = addmod(mulmod(a0, b1, q), mulmod(a1, b0, q), q);
      out[((size_t)2 * nl + k) * N + i] = mulmod(a1, b1, q);
    }
  }
  return 0;
}

/* Rescale (Appendix A): floor(x / q_l) rounded, i.e.
 * out_i = (x_i - [x]_{q_l}) q_l^{-1} mod q_i, with [.] centred. */
oc_ct *oc_rescale(const oc_ctx *c, const oc_ct *a) {
  if (a->qp || a->level < 1) return NULL;
  u64 N = c->N;
  int l = a->level;
  u64 ql = c->mods[l];
  oc_ct *r = ct_new(c, l - 1, 0, a->scale / (double)ql);
  u64 *top = alloc_u64(N);
  for (int p = 0; p < 2; p++) {
    memcpy(top, poly(c, a, p, l), sizeof(u64) * N);
    oc_intt(c, l, top);
#pragma omp parallel for schedule(dynamic)
    for (int k = 0; k < l; k++) {
      u64 q = c->mods[k];
      u64 *t = alloc_u64(N);
      for (u64 i = 0; i < N; i++) {
        i64 centred = top[i] > ql / 2 ? (i64)top[i] - (i64)ql : (i64)top[i];
        t[i] = smod(centred, q);
      }
      oc_ntt(c, k, t);
      u64 inv = invmod(ql % q, q);
      for (u64 i = 0; i < N; i++) poly(c, r, p, k)[i] = mulmod(submod(poly(c, a, p, k)[i], t[i], q), inv, q);
      free(t);
    }
  }
  free(top);
  return r;
}

/* drop to a lower level without rescaling (keep the first level'+1 limbs) */
oc_ct *oc_drop(const oc_ctx *c, const oc_ct *a, int level) {
  if (a->qp || level > a->level || level < 0) return NULL;
  oc_ct *r = ct_new(c, level, 0, a->scale);
  for (int p = 0; p < 2; p++)
    for (int k = 0; k <= level; k++) memcpy(poly(c, r, p, k), poly(c, a, p, k), sizeof(u64) * c->N);
  return r;
}

/* ------------------------------------------------------------------------ */
/* Key switching pieces (section 3.3.1 hoisting; Appendix A KeySwitch).      */
/* ------------------------------------------------------------------------ */
/* Fast basis conversion of coefficient-domain residues x_i (i in src) to the
 * modulus t:  sum_i [x_i (D/q_i)^{-1}]_{q_i} (D/q_i)  mod t,  D = prod src. */
static void fbc(const oc_ctx *c, const u64 *const *x, const int *src, int ns, int tmod, u64 *out) {
  u64 N = c->N, t = c->mods[tmod];
  u64 hat_inv[MAXMOD], hat_t[MAXMOD];
  for (int a = 0; a < ns; a++) {
    u64 qa = c->mods[src[a]];
    u64 h = 1, ht = 1;
    for (int b = 0; b < ns; b++) {
      if (b == a) continue;
      h = mulmod(h, c->mods[src[b]] % qa, qa);
      ht = mulmod(ht, c->mods[src[b]] % t, t);
    }
    hat_inv[a] = invmod(h, qa);
    hat_t[a] = ht;
  }
  for (u64 i = 0; i < N; i++) {
    u64 acc = 0;
    for (int a = 0; a < ns; a++) {
      u64 y = mulmod(x[a][i], hat_inv[a], c->mods[src[a]]);
      acc = addmod(acc, mulmod(y % t, hat_t[a], t), t);
    }
    out[i] = acc;
  }
}

/* Decompose (ModUp): d (NTT domain over Q_level) -> beta_l digits, each over
 * Q_level and P, NTT domain: u64[beta_l][level+1+alpha][N].  Limbs of the
 * digit's own primes are the input residues themselves. */
int oc_beta_at(const oc_ctx *c, int level) { return (level + c->alpha) / c->alpha; }

u64 *oc_decompose(const oc_ctx *c, const u64 *d, int level) {
  u64 N = c->N;
  int nq = level + 1, nqp = nq + c->alpha, beta = oc_beta_at(c, level);
  u64 *coef = alloc_u64((size_t)nq * N);
  memcpy(coef, d, sizeof(u64) * nq * N);
  int idx[MAXMOD];
  for (int k = 0; k < nq; k++) idx[k] = k;
  intt_limbs(c, coef, idx, nq);
  u64 *out = alloc_u64((size_t)beta * nqp * N);
  for (int j = 0; j < beta; j++) {
    int src[MAXMOD], ns = 0;
    for (int k = j * c->alpha; k < (j + 1) * c->alpha && k < nq; k++) src[ns++] = k;
    const u64 *xs[MAXMOD];
    for (int a = 0; a < ns; a++) xs[a] = coef + (size_t)src[a] * N;
#pragma omp parallel for schedule(dynamic)
    for (int pos = 0; pos < nqp; pos++) {
      u64 *o = out + ((size_t)j * nqp + pos) * N;
      int m = qp_mod_index(c, level, pos);
      int own = pos < nq && pos / c->alpha == j;
      if (own) {
        memcpy(o, d + (size_t)pos * N, sizeof(u64) * N);
      } else {
        fbc(c, xs, src, ns, m, o);
        oc_ntt(c, m, o);
      }
    }
  }
  free(coef);
  return out;
}

/* Fixed-width unsigned big integers (little-endian 64-bit words), enough for
 * products of up to four 61-bit primes. */
#define BW 5
typedef struct { u64 w[BW]; } big;
static big big_u64(u64 v) { big r; memset(&r, 0, sizeof r); r.w[0] = v; return r; }
static big big_mul_u64(big a, u64 b) {
  big r;
  u128 carry = 0;
  for (int k = 0; k < BW; k++) {
    u128 t = (u128)a.w[k] * b + carry;
    r.w[k] = (u64)t;
    carry = t >> 64;
  }
  return r;
}
static big big_add(big a, big b) {
  big r;
  u128 carry = 0;
  for (int k = 0; k < BW; k++) {
    u128 t = (u128)a.w[k] + b.w[k] + carry;
    r.w[k] = (u64)t;
    carry = t >> 64;
  }
  return r;
}
static big big_sub(big a, big b) { /* a >= b */
  big r;
  u64 borrow = 0;
  for (int k = 0; k < BW; k++) {
    u64 t = a.w[k] - b.w[k] - borrow;
    borrow = (a.w[k] < b.w[k]) || (a.w[k] - b.w[k] < borrow);
    r.w[k] = t;
  }
  return r;
}
static int big_cmp(big a, big b) {
  for (int k = BW - 1; k >= 0; k--) {
    if (a.w[k] != b.w[k]) return a.w[k] < b.w[k] ? -1 : 1;
  }
  return 0;
}
static u64 big_mod_u64(big a, u64 q) {
  u128 r = 0;
  for (int k = BW - 1; k >= 0; k--) r = ((r << 64) | a.w[k]) % q;
  return (u64)r;
}

/* Exact rounded division by the product D of some limbs of x (NTT domain):
 * the source limbs sit at positions spos[] of x with moduli smod[]; for the
 * moduli q_0..q_{nout-1} (positions 0..nout-1)
 *   out_i = (x_i - [x]_D) D^{-1} mod q_i,
 * with [x]_D the exact centred residue of x modulo D, reconstructed by CRT
 * from the source limbs.  x - [x]_D is divisible by D, so this is
 * round(x / D) (D is odd: no ties). */
static void divide_round_poly(const oc_ctx *c, const u64 *x, const int *spos, const int *smod, int ns, int nout,
                              u64 *out) {
  u64 N = c->N;
  u64 *pc = alloc_u64((size_t)ns * N);
  int pidx[MAXMOD];
  for (int k = 0; k < ns; k++) {
    pidx[k] = smod[k];
    memcpy(pc + (size_t)k * N, x + (size_t)spos[k] * N, sizeof(u64) * N);
  }
  intt_limbs(c, pc, pidx, ns);
  /* CRT constants: D, D/d_k and (D/d_k)^{-1} mod d_k */
  big D = big_u64(1), H[MAXMOD];
  u64 Hinv[MAXMOD];
  for (int k = 0; k < ns; k++) D = big_mul_u64(D, c->mods[smod[k]]);
  for (int k = 0; k < ns; k++) {
    u64 dk = c->mods[smod[k]];
    H[k] = big_u64(1);
    for (int m = 0; m < ns; m++)
      if (m != k) H[k] = big_mul_u64(H[k], c->mods[smod[m]]);
    Hinv[k] = invmod(big_mod_u64(H[k], dk), dk);
  }
  /* centred residue, kept as (magnitude, sign) per coefficient */
  big *mag = (big *)malloc(sizeof(big) * N);
  char *neg = (char *)malloc(N);
#pragma omp parallel for schedule(static)
  for (u64 t = 0; t < N; t++) {
    big S = big_u64(0);
    for (int k = 0; k < ns; k++) {
      u64 dk = c->mods[smod[k]];
      S = big_add(S, big_mul_u64(H[k], mulmod(pc[(size_t)k * N + t], Hinv[k], dk)));
    }
    while (big_cmp(S, D) >= 0) S = big_sub(S, D);
    big twoS = big_add(S, S);
    if (big_cmp(twoS, D) > 0) { mag[t] = big_sub(D, S); neg[t] = 1; }
    else { mag[t] = S; neg[t] = 0; }
  }
#pragma omp parallel for schedule(dynamic)
  for (int i = 0; i < nout; i++) {
    u64 q = c->mods[i];
    u64 *y = alloc_u64(N);
    for (u64 t = 0; t < N; t++) {
      u64 r = big_mod_u64(mag[t], q);
      y[t] = neg[t] ? (r ? q - r : 0) : r;
    }
    oc_ntt(c, i, y);
    u64 dinv = 1;
    for (int k = 0; k < ns; k++) dinv = mulmod(dinv, c->mods[smod[k]] % q, q);
    dinv = invmod(dinv, q);
    for (u64 t = 0; t < N; t++)
      out[(size_t)i * N + t] = mulmod(submod(x[(size_t)i * N + t], y[t], q), dinv, q);
    free(y);
  }
  free(pc);
  free(mag);
  free(neg);
}

/* ModDown (Appendix A, KeySwitch): x in R_{Q_l P} (NTT domain, l+1+alpha
 * limbs) -> round(x / P) in R_{Q_l}: the division above with the P limbs as
 * sources. */
static void moddown_poly(const oc_ctx *c, const u64 *x, int level, u64 *out) {
  int spos[MAXMOD], smod[MAXMOD];
  for (int k = 0; k < c->alpha; k++) {
    spos[k] = level + 1 + k;
    smod[k] = c->L + 1 + k;
  }
  divide_round_poly(c, x, spos, smod, c->alpha, level + 1, out);
}

/* ModDown and the Rescale after it as one rounding (a variant of the paper's
 * two): x in R_{Q_l P} -> round(x / (P q_l)) in R_{Q_{l-1}}, the division
 * above with q_l and the P limbs as sources.  It differs from
 * Rescale(ModDown(x)) = round(round(x / P) / q_l) by at most one in a
 * coefficient. */
static void moddown_rescale_poly(const oc_ctx *c, const u64 *x, int level, u64 *out) {
  int spos[MAXMOD], smod[MAXMOD];
  spos[0] = level;
  smod[0] = level;
  for (int k = 0; k < c->alpha; k++) {
    spos[k + 1] = level + 1 + k;
    smod[k + 1] = c->L + 1 + k;
  }
  divide_round_poly(c, x, spos, smod, c->alpha + 1, level, out);
}

oc_ct *oc_moddown_rescale(const oc_ctx *c, const oc_ct *a) {
  if (!a->qp || a->level < 1) return NULL;
  oc_ct *r = ct_new(c, a->level - 1, 0, a->scale / (double)c->mods[a->level]);
  for (int p = 0; p < 2; p++) moddown_rescale_poly(c, poly(c, a, p, 0), a->level, poly(c, r, p, 0));
  return r;
}

oc_ct *oc_moddown(const oc_ctx *c, const oc_ct *a) {
  if (!a->qp) return NULL;
  oc_ct *r = ct_new(c, a->level, 0, a->scale);
  for (int p = 0; p < 2; p++) moddown_poly(c, poly(c, a, p, 0), a->level, poly(c, r, p, 0));
  return r;
}

/* MultSum with optional permutation: for both key halves,
 *   acc_t = sum_j pi_g(d_j)_t * swk_j,t   over t in Q_l and P. */
static void multsum(const oc_ctx *c, const u64 *digits, int level, u64 g, const oc_key *key,
                    u64 *out /* [2][nqp][N] */) {
  u64 N = c->N;
  int nq = level + 1, nqp = nq + c->alpha, beta = oc_beta_at(c, level), nm = c->nmods;
#pragma omp parallel for schedule(dynamic)
  for (int pos = 0; pos < nqp; pos++) {
    int m = qp_mod_index(c, level, pos);
    u64 q = c->mods[m];
    u64 *perm = alloc_u64(N);
    u64 *acc0 = out + ((size_t)0 * nqp + pos) * N;
    u64 *acc1 = out + ((size_t)1 * nqp + pos) * N;
    for (u64 i = 0; i < N; i++) { acc0[i] = 0; acc1[i] = 0; }
    for (int j = 0; j < beta; j++) {
      const u64 *dj = digits + ((size_t)j * nqp + pos) * N;
      if (g != 1) oc_automorph_ntt(c, g, dj, perm);
      else memcpy(perm, dj, sizeof(u64) * N);
      const u64 *kb = key->data + (((size_t)j * 2 + 0) * nm + m) * N;
      const u64 *ka = key->data + (((size_t)j * 2 + 1) * nm + m) * N;
      for (u64 i = 0; i < N; i++) {
        acc0[i] = addmod(acc0[i], mulmod(perm[i], kb[i], q), q);
        acc1[i] = addmod(acc1[i], mulmod(perm[i], ka[i], q), q);
      }
    }
    free(perm);
  }
}

/* KeySwitch(d, swk) = ModDown(<Decompose(d), swk>), d over Q_level (NTT). */
static int keyswitch(const oc_ctx *c, const u64 *d, int level, const oc_key *key, u64 *out /* [2][l+1][N] */) {
  u64 N = c->N;
  int nq = level + 1, nqp = nq + c->alpha;
  u64 *dig = oc_decompose(c, d, level);
  u64 *acc = alloc_u64((size_t)2 * nqp * N);
  multsum(c, dig, level, 1, key, acc);
  moddown_poly(c, acc, level, out);
  moddown_poly(c, acc + (size_t)nqp * N, level, out + (size_t)nq * N);
  free(dig); free(acc);
  return 0;
}

/* Mult with relinearisation: (d0, d1) + KeySwitch(d2, rlk). */
oc_ct *oc_relin(const oc_ctx *c, const u64 *t3, int level, double scale) {
  const oc_key *rlk = find_key(c, 0);
  if (!rlk) return NULL;
  u64 N = c->N;
  int nq = level + 1;
  u64 *ks = alloc_u64((size_t)2 * nq * N);
  keyswitch(c, t3 + (size_t)2 * nq * N, level, rlk, ks);
  oc_ct *r = ct_new(c, level, 0, scale);
  for (int p = 0; p < 2; p++)
    for (int k = 0; k < nq; k++) {
      u64 q = c->mods[k];
      for (u64 i = 0; i < N; i++)
        poly(c, r, p, k)[i] = addmod(t3[((size_t)p * nq + k) * N + i], ks[((size_t)p * nq + k) * N + i], q);
    }
  free(ks);
  return r;
}

oc_ct *oc_mult(const oc_ctx *c, const oc_ct *a, const oc_ct *b) {
  if (!same_shape(a, b) || a->qp) return NULL;
  u64 *t3 = alloc_u64((size_t)3 * a->nlimbs * c->N);
  oc_tensor(c, a, b, t3);
  oc_ct *r = oc_relin(c, t3, a->level, a->scale * b->scale);
  free(t3);
  return r;
}

/* Hoisted rotation left in R_{Q_l P} (section 3.3.1):
 *   HR(c, g) = (P pi_g(c0) + sum_j pi_g(d_j) swk_j.b,  sum_j pi_g(d_j) swk_j.a)
 * with the digits d = Decompose(c1) computed once by the caller.
 * For g = 1 (no rotation) it is the P-lift (P c0, P c1). */
static oc_ct *hoisted_rot(const oc_ctx *c, const oc_ct *x, const u64 *digits, u64 g, int *err) {
  u64 N = c->N;
  int level = x->level, nq = level + 1, nqp = nq + c->alpha;
  oc_ct *r = ct_new(c, level, 1, x->scale);
  u64 *perm = alloc_u64(N);
  if (g == 1) {
    for (int p = 0; p < 2; p++)
      for (int k = 0; k < nq; k++) {
        u64 q = c->mods[k], pm = 1;
        for (int a = 0; a < c->alpha; a++) pm = mulmod(pm, c->mods[c->L + 1 + a] % q, q);
        for (u64 i = 0; i < N; i++) poly(c, r, p, k)[i] = mulmod(poly(c, x, p, k)[i], pm, q);
      }
    free(perm);
    return r;
  }
  const oc_key *key = find_key(c, g);
  if (!key) { *err = -4; oc_ct_free(r); free(perm); return NULL; }
  multsum(c, digits, level, g, key, r->d);
  for (int k = 0; k < nq; k++) {
    u64 q = c->mods[k], pm = 1;
    for (int a = 0; a < c->alpha; a++) pm = mulmod(pm, c->mods[c->L + 1 + a] % q, q);
    oc_automorph_ntt(c, g, poly(c, x, 0, k), perm);
    for (u64 i = 0; i < N; i++) poly(c, r, 0, k)[i] = addmod(poly(c, r, 0, k)[i], mulmod(perm[i], pm, q), q);
  }
  (void)nqp;
  free(perm);
  return r;
}

oc_ct *oc_hoisted_rotate(const oc_ctx *c, const oc_ct *x, i64 step) {
  if (x->qp) return NULL;
  u64 g = oc_galois_of_step(c, step);
  u64 *dig = g == 1 ? NULL : oc_decompose(c, poly(c, x, 1, 0), x->level);
  int err = 0;
  oc_ct *r = hoisted_rot(c, x, dig, g, &err);
  free(dig);
  return r;
}

/* The same with the digits Decompose(c1) given by the caller (so that the
 * key inner product can be timed on its own). */
oc_ct *oc_hoisted_rotate_digits(const oc_ctx *c, const oc_ct *x, const u64 *digits, i64 step) {
  if (x->qp) return NULL;
  int err = 0;
  return hoisted_rot(c, x, digits, oc_galois_of_step(c, step), &err);
}

/* OpenMP threads of the oracle's loops over limbs (timing runs only) */
void oc_set_threads(int n) { omp_set_num_threads(n > 0 ? n : 1); }
int oc_get_threads(void) { return omp_get_max_threads(); }

/* Rot(c, k) = ModDown(HR(c, 5^k)). */
oc_ct *oc_rotate(const oc_ctx *c, const oc_ct *x, i64 step) {
  oc_ct *h = oc_hoisted_rotate(c, x, step);
  if (!h) return NULL;
  oc_ct *r = oc_moddown(c, h);
  oc_ct_free(h);
  return r;
}

/* ------------------------------------------------------------------------ */
/* Homomorphic linear transforms by double-hoisted BSGS                      */
/* (Eq. 2, Eq. 3', hoisting and double hoisting in section 3.3.1).           */
/* ------------------------------------------------------------------------ */
/* A linear transform on the n^2-vector given as a permutation with optional
 * weights: output index t takes w[t] * input[perm[t]].  Its l-th diagonal is
 * u_l[t] = w[t] if perm[t] = t + l (mod n^2), else 0. */
typedef struct {
  int n2;           /* vector length n^2 */
  const int *perm;  /* [n2] */
  const double *w;  /* [n2] weights (NULL = all ones) */
} lt_perm;

static i64 pmod_i(i64 a, i64 m) { return ((a % m) + m) % m; }

/* diagonal u_l, pre-rotated by -shift: out[t] = u_l[t - shift]
 * (perm[s] < 0 marks an all-zero row) */
static int diag_vec(const lt_perm *U, i64 l, i64 shift, double *out) {
  int nz = 0;
  i64 n2 = U->n2;
  for (i64 t = 0; t < n2; t++) {
    i64 s = pmod_i(t - shift, n2);
    double v = 0.0;
    if (U->perm[s] >= 0 && pmod_i((i64)U->perm[s] - s, n2) == pmod_i(l, n2)) v = U->w ? U->w[s] : 1.0;
    out[t] = v;
    if (v != 0.0) nz = 1;
  }
  return nz;
}

/* pt over the QP limbs of an element at `level`, as integer coefficients */
static void pt_int(const oc_ctx *c, const double *vec, int n2, double scale, i64 *m) {
  oc_encode(c, vec, n2, scale, m);
}

/* acc += pt (.) h, all over Q_l P */
static void qp_pmult_acc(const oc_ctx *c, oc_ct *acc, const oc_ct *h, const i64 *m) {
  int nl = h->nlimbs, idx[MAXMOD];
  for (int k = 0; k < nl; k++) idx[k] = limb_mod(c, h, k);
  u64 *mn = alloc_u64((size_t)nl * c->N);
  poly_from_int(c, m, idx, nl, mn);
  for (int p = 0; p < 2; p++)
    for (int k = 0; k < nl; k++) {
      u64 q = c->mods[idx[k]];
      for (u64 i = 0; i < c->N; i++)
        poly(c, acc, p, k)[i] =
            addmod(poly(c, acc, p, k)[i], mulmod(poly(c, h, p, k)[i], mn[(size_t)k * c->N + i], q), q);
    }
  free(mn);
}

typedef struct {
  int decompose, multsum, moddown, rescale, pmult;
} oc_counts;
static oc_counts g_counts;
void oc_counts_reset(void) { memset(&g_counts, 0, sizeof g_counts); }
void oc_counts_get(int *out5) {
  out5[0] = g_counts.decompose; out5[1] = g_counts.multsum; out5[2] = g_counts.moddown;
  out5[3] = g_counts.rescale; out5[4] = g_counts.pmult;
}

/* U m via double-hoisted BSGS with indices a (n1 i + j), j in [0, n1),
 * i in [i_lo, i_hi); diagonals encoded at scale pt_scale; one Rescale. */
/* With 2 <= n1p < n1 the baby steps follow the simple key substitution of
 * section 4.2.1: only the keys a j', 0 < j' < n1p, of the inner loop exist.
 * The steps j = b n1p + j' are taken in blocks b, HR(x_b, a j') from the
 * block's own Decompose, where x_0 = x and x_b = Rot(x_{b-1}, a n1p) is
 * reached with those keys: ModDown(HR(x_{b-1}, a (n1p - 1))), then Rot by a. */
static oc_ct *lintrans(const oc_ctx *c, const oc_ct *x, const lt_perm *U, i64 a, int n1, int i_lo,
                       int i_hi, int n1p, int *err) {
  u64 N = c->N;
  int level = x->level;
  if (level < 1) { *err = -2; return NULL; }
  /* diagonals encoded at scale q_l: the closing rescale by q_l gives back
   * exactly the input scale */
  double pt_scale = (double)c->mods[level];
  int blk = (n1p >= 2 && n1p < n1) ? n1p : n1;
  oc_ct *xb = NULL; /* base of the current block when b > 0 */
  u64 *dig = NULL;
  oc_ct **baby = (oc_ct **)calloc(n1, sizeof(oc_ct *));
  double *vec = (double *)malloc(sizeof(double) * U->n2);
  i64 *m = (i64 *)malloc(sizeof(i64) * N);
  /* only baby steps some giant step actually uses are formed */
  int *used = (int *)calloc(n1, sizeof(int));
  for (int i = i_lo; i < i_hi; i++)
    for (int j = 0; j < n1; j++)
      if (diag_vec(U, a * ((i64)n1 * i + j), a * (i64)n1 * i, vec)) used[j] = 1;
  for (int b = 0; b * blk < n1; b++) {
    const oc_ct *base = b == 0 ? x : xb;
    int more = (b + 1) * blk < n1, jl = b * blk + blk - 1;
    dig = oc_decompose(c, poly(c, base, 1, 0), level);
    g_counts.decompose++;
    for (int jp = 0; jp < blk && b * blk + jp < n1; jp++) {
      int j = b * blk + jp;
      if (!used[j] && !(more && j == jl)) continue;
      baby[j] = hoisted_rot(c, base, dig, oc_galois_of_step(c, a * jp), err);
      if (!baby[j]) goto fail;
      if (jp) g_counts.multsum++;
    }
    free(dig);
    dig = NULL;
    if (more) {
      oc_ct *y = oc_moddown(c, baby[jl]);
      g_counts.moddown++;
      if (!used[jl]) { oc_ct_free(baby[jl]); baby[jl] = NULL; }
      oc_ct *nb = oc_rotate(c, y, a);
      g_counts.decompose++; g_counts.multsum++; g_counts.moddown++;
      oc_ct_free(y);
      oc_ct_free(xb);
      xb = nb;
      if (!xb) { *err = -4; goto fail; }
    }
  }
  oc_ct_free(xb);
  xb = NULL;
  oc_ct *acc = ct_new(c, level, 1, x->scale * pt_scale);
  for (int i = i_lo; i < i_hi; i++) {
    oc_ct *inner = NULL;
    for (int j = 0; j < n1; j++) {
      i64 l = a * ((i64)n1 * i + j);
      if (!diag_vec(U, l, a * (i64)n1 * i, vec)) continue;
      pt_int(c, vec, U->n2, pt_scale, m);
      if (!inner) inner = ct_new(c, level, 1, x->scale * pt_scale);
      qp_pmult_acc(c, inner, baby[j], m);
      g_counts.pmult++;
    }
    if (!inner) continue;
    if (i == 0) {
      add_into(c, acc, inner);
    } else {
      oc_ct *t = oc_moddown(c, inner);
      g_counts.moddown++;
      u64 *d2 = oc_decompose(c, poly(c, t, 1, 0), level);
      g_counts.decompose++;
      oc_ct *h = hoisted_rot(c, t, d2, oc_galois_of_step(c, a * (i64)n1 * i), err);
      g_counts.multsum++;
      free(d2);
      oc_ct_free(t);
      if (!h) { oc_ct_free(inner); oc_ct_free(acc); goto fail; }
      add_into(c, acc, h);
      oc_ct_free(h);
    }
    oc_ct_free(inner);
  }
  oc_ct *md = oc_moddown(c, acc);
  g_counts.moddown++;
  oc_ct_free(acc);
  oc_ct *r = oc_rescale(c, md);
  g_counts.rescale++;
  oc_ct_free(md);
  if (r) r->scale = x->scale;
  for (int j = 0; j < n1; j++) oc_ct_free(baby[j]);
  free(baby); free(vec); free(m); free(dig); free(used);
  return r;
fail:
  for (int j = 0; j < n1; j++) oc_ct_free(baby[j]);
  oc_ct_free(xb);
  free(baby); free(vec); free(m); free(dig); free(used);
  return NULL;
}

/* ------------------------------------------------------------------------ */
/* Jiang's permutations on row-major n x n matrices (Eq. 4; Eq. 5, Eq. 6)     */
/*   sigma(A)_{i,j} = A_{i,(i+j) mod n}        (Z)                           */
/*   tau(B)_{i,j}   = B_{(i+j) mod n, j}       (T)                           */
/*   phi^k(A)_{i,j} = A_{i,(j+k) mod n}        (C^k)                         */
/*   psi^k(B)_{i,j} = B_{(i+k) mod n, j}       (R^k)                         */
/*   transpose: A^T_{i,j} = A_{j,i}            (G)                           */
/* ------------------------------------------------------------------------ */
static int *perm_sigma(int n) {
  int *p = (int *)malloc(sizeof(int) * n * n);
  for (int i = 0; i < n; i++)
    for (int j = 0; j < n; j++) p[i * n + j] = i * n + (i + j) % n;
  return p;
}
static int *perm_tau(int n) {
  int *p = (int *)malloc(sizeof(int) * n * n);
  for (int i = 0; i < n; i++)
    for (int j = 0; j < n; j++) p[i * n + j] = ((i + j) % n) * n + j;
  return p;
}
static int *perm_transpose(int n) {
  int *p = (int *)malloc(sizeof(int) * n * n);
  for (int i = 0; i < n; i++)
    for (int j = 0; j < n; j++) p[i * n + j] = j * n + i;
  return p;
}

void oc_perm(int which, int n, int *out) {
  int *p = which == 0 ? perm_sigma(n) : which == 1 ? perm_tau(n) : perm_transpose(n);
  memcpy(out, p, sizeof(int) * n * n);
  free(p);
}

/* BSGS giant-step ranges (reading of Eq. 3': indices a (n1 i + j)) */
static int ceil_div(int a, int b) { return (a + b - 1) / b; }

/* sigma (Z): a = 1, giants i in [-n2, n2) */
oc_ct *oc_lt_sigma(const oc_ctx *c, const oc_ct *x, int n, int n1, int *err) {
  int *p = perm_sigma(n);
  lt_perm U = {n * n, p, NULL};
  int n2 = ceil_div(n, n1);
  oc_ct *r = lintrans(c, x, &U, 1, n1, -n2, n2, 0, err);
  free(p);
  return r;
}
/* tau (T): a = n, giants i in [0, n2) */
oc_ct *oc_lt_tau(const oc_ctx *c, const oc_ct *x, int n, int n1, int *err) {
  int *p = perm_tau(n);
  lt_perm U = {n * n, p, NULL};
  int n2 = ceil_div(n, n1);
  oc_ct *r = lintrans(c, x, &U, n, n1, 0, n2, 0, err);
  free(p);
  return r;
}
/* transposition (G): a = n - 1, giants i in [-n2, n2); optional uniform weight */
oc_ct *oc_lt_transpose(const oc_ctx *c, const oc_ct *x, int n, int n1, double weight, int *err) {
  int *p = perm_transpose(n);
  double *w = NULL;
  if (weight != 1.0) {
    w = (double *)malloc(sizeof(double) * n * n);
    for (int t = 0; t < n * n; t++) w[t] = weight;
  }
  lt_perm U = {n * n, p, w};
  int n2 = ceil_div(n, n1);
  oc_ct *r = lintrans(c, x, &U, n - 1, n1, -n2, n2, 0, err);
  free(p); free(w);
  return r;
}

/* ------------------------------------------------------------------------ */
/* Diagonal convergence decomposition (section 4.2: Definition 4, Theorem 2, */
/* Algorithms DCDforZ and DCDforT).                                          */
/*                                                                           */
/* A permutation transform (output t takes input perm[t]) is written as a   */
/* product L R_m ... R_1 (R_1 applied first).  Following one 1-entry of the */
/* matrix with remaining diagonal k, each right factor moves it by r(k) and */
/* keeps the column (Definition 4); the left factor takes the rest:          */
/*   Z: |k| >= n'  -> r = sign(k) n',  else 0   (Z split into k >= 0, k < 0) */
/*   T: k = i n, i > n' -> r = n' n,    else 0                                */
/* with ceil((n-1)/n') - 1 right factors.                                    */
/* ------------------------------------------------------------------------ */
typedef struct {
  int n2;
  int *perm; /* -1: zero row */
  i64 a;     /* BSGS stride */
  int n1, i_lo, i_hi;
} oc_factor;

static i64 floor_div_i(i64 a, i64 b) { return a >= 0 ? a / b : -((-a + b - 1) / b); }

enum { DCD_Z1 = 0, DCD_Z2 = 1, DCD_T = 2 };

/* factors in application order; returns their count, -1 if a factor would
 * not be a partial permutation */
static int dcd_chain(int n, const int *perm, int which, int nprime, int n1, oc_factor *out) {
  int n2 = n * n;
  int iters = ceil_div(n - 1, nprime) - 1;
  i64 *pos = (i64 *)malloc(sizeof(i64) * n2), *k = (i64 *)malloc(sizeof(i64) * n2);
  char *sel = (char *)calloc(n2, 1);
  for (int t = 0; t < n2; t++) {
    i64 kk = which == DCD_T ? pmod_i((i64)perm[t] - t, n2) : (i64)perm[t] - t;
    if (which == DCD_Z1 && kk < 0) continue;
    if (which == DCD_Z2 && kk >= 0) continue;
    sel[t] = 1;
    pos[t] = perm[t];
    k[t] = kk;
  }
  i64 dnz = which == DCD_Z1 ? nprime : which == DCD_Z2 ? -nprime : (i64)nprime * n;
  for (int j = 0; j < iters; j++) {
    oc_factor *f = &out[j];
    f->n2 = n2;
    f->perm = (int *)malloc(sizeof(int) * n2);
    for (int t = 0; t < n2; t++) f->perm[t] = -1;
    for (int t = 0; t < n2; t++) {
      if (!sel[t]) continue;
      i64 d;
      if (which == DCD_T) d = (k[t] / n > nprime) ? dnz : 0;
      else d = (k[t] >= nprime || k[t] <= -nprime) ? dnz : 0;
      i64 np = pmod_i(pos[t] - d, n2);
      if (f->perm[np] != -1) { free(pos); free(k); free(sel); return -1; }
      f->perm[np] = (int)pos[t];
      pos[t] = np;
      k[t] -= d;
    }
    f->a = dnz;
    f->n1 = 2;
    f->i_lo = 0;
    f->i_hi = 1;
  }
  oc_factor *lf = &out[iters];
  lf->n2 = n2;
  lf->perm = (int *)malloc(sizeof(int) * n2);
  i64 a = which == DCD_T ? n : 1, kmin = 0, kmax = 0;
  int first = 1;
  for (int t = 0; t < n2; t++) {
    lf->perm[t] = sel[t] ? (int)pos[t] : -1;
    if (!sel[t]) continue;
    i64 kk = k[t] / a;
    if (first || kk < kmin) kmin = kk;
    if (first || kk > kmax) kmax = kk;
    first = 0;
  }
  lf->a = a;
  lf->n1 = n1;
  lf->i_lo = (int)floor_div_i(kmin, n1);
  lf->i_hi = (int)floor_div_i(kmax, n1) + 1;
  free(pos); free(k); free(sel);
  return iters + 1;
}

/* exported for the planner pins: factor count and each factor's perm */
int oc_dcd_factors(int n, int which, int nprime, int n1, int *perms /* [maxf][n*n] */, long long *geom /* [maxf][4] */,
                   int maxf) {
  int *p = which == DCD_T ? perm_tau(n) : perm_sigma(n);
  oc_factor f[64];
  int nf = dcd_chain(n, p, which, nprime, n1, f);
  free(p);
  if (nf < 0) return -1;
  for (int j = 0; j < nf; j++) {
    if (j < maxf) {
      memcpy(perms + (size_t)j * n * n, f[j].perm, sizeof(int) * n * n);
      geom[4 * j] = f[j].a; geom[4 * j + 1] = f[j].n1; geom[4 * j + 2] = f[j].i_lo; geom[4 * j + 3] = f[j].i_hi;
    }
    free(f[j].perm);
  }
  return nf;
}

static oc_ct *apply_chain(const oc_ctx *c, const oc_ct *x, const oc_factor *f, int nf, int *err) {
  oc_ct *cur = oc_ct_copy(c, x);
  for (int j = 0; j < nf && cur; j++) {
    lt_perm U = {f[j].n2, f[j].perm, NULL};
    oc_ct *nx = lintrans(c, cur, &U, f[j].a, f[j].n1, f[j].i_lo, f[j].i_hi, 0, err);
    oc_ct_free(cur);
    cur = nx;
  }
  return cur;
}

/* sigma (Z) of Algorithm DMatrixMult: Z1 chain + Z2 chain when n' < n-1 */
static oc_ct *sigma_dcd(const oc_ctx *c, const oc_ct *x, int n, int n1, int nprime, int *err) {
  if (nprime >= n - 1) return oc_lt_sigma(c, x, n, n1, err);
  int *p = perm_sigma(n);
  oc_factor f1[64], f2[64];
  int c1 = dcd_chain(n, p, DCD_Z1, nprime, n1, f1), c2 = dcd_chain(n, p, DCD_Z2, nprime, n1, f2);
  free(p);
  if (c1 < 0 || c2 < 0) { *err = -1; return NULL; }
  oc_ct *a1 = apply_chain(c, x, f1, c1, err);
  oc_ct *a2 = apply_chain(c, x, f2, c2, err);
  oc_ct *r = (a1 && a2) ? oc_add(c, a1, a2) : NULL;
  oc_ct_free(a1); oc_ct_free(a2);
  for (int j = 0; j < c1; j++) free(f1[j].perm);
  for (int j = 0; j < c2; j++) free(f2[j].perm);
  return r;
}

/* tau (T): one chain when n' < n-1 */
static oc_ct *tau_dcd(const oc_ctx *c, const oc_ct *x, int n, int n1, int nprime, int *err) {
  if (nprime >= n - 1) return oc_lt_tau(c, x, n, n1, err);
  int *p = perm_tau(n);
  oc_factor f[64];
  int nf = dcd_chain(n, p, DCD_T, nprime, n1, f);
  free(p);
  if (nf < 0) { *err = -1; return NULL; }
  oc_ct *r = apply_chain(c, x, f, nf, err);
  for (int j = 0; j < nf; j++) free(f[j].perm);
  return r;
}

/* ------------------------------------------------------------------------ */
/* The homomorphic matrix product (Eq. 4; Algorithm DMatrixMult; hoisted     */
/* column / row shifts of section 4.1.1).                                    */
/* ------------------------------------------------------------------------ */
static void col_mask(int n, int k, int second, double *out) {
  for (int i = 0; i < n; i++)
    for (int j = 0; j < n; j++) {
      int in_first = j < n - k;
      out[i * n + j] = (second ? !in_first : in_first) ? 1.0 : 0.0;
    }
}

/* A side: A_k = C^k Z a for k < n.  Bases B_b = Rot(B_{b-1}, n1z) from
 * B_0 = Z a and B'_0 = Rot(Z a, -n); for k = b n1z + r:
 *   A_k = Rescale(ModDown(m_k (.) HR(B_b, r) + m'_k (.) HR(B'_b, r))). */
/* (fused: one rounding by P q_l in place of ModDown then Rescale) */
/* Z (kind 0) or T (kind 1) of a d x d matrix ciphertext, decomposed (section
 * 4.2) when 0 < nprime < n - 1: the transform alone, as the product's sides
 * start with it */
/* Z (kind 0) or T (kind 1) by dh-BSGS with the simple key substitution of
 * the baby steps (section 4.2.1), prefix n1p */
oc_ct *oc_lt_smpkeysub(const oc_ctx *c, const oc_ct *x, int kind, int n, int n1, int n1p, int *err) {
  *err = 0;
  if (kind < 0 || kind > 1 || n1p == 1) { *err = -1; return NULL; }
  int *p = kind == 0 ? perm_sigma(n) : perm_tau(n);
  lt_perm U = {n * n, p, NULL};
  int n2 = ceil_div(n, n1);
  oc_ct *r = kind == 0 ? lintrans(c, x, &U, 1, n1, -n2, n2, n1p, err) : lintrans(c, x, &U, n, n1, 0, n2, n1p, err);
  free(p);
  return r;
}

oc_ct *oc_lt_dcd(const oc_ctx *c, const oc_ct *x, int kind, int n, int n1, int nprime, int *err) {
  *err = 0;
  if (kind == 0) return sigma_dcd(c, x, n, n1, nprime, err);
  if (kind == 1) return tau_dcd(c, x, n, n1, nprime, err);
  *err = -1;
  return NULL;
}

static oc_ct **side_a(const oc_ctx *c, const oc_ct *ca, int n, int n1z, int npz, int fused, int *err) {
  u64 N = c->N;
  int n2sq = n * n;
  oc_ct *A0 = sigma_dcd(c, ca, n, n1z, npz, err);
  if (!A0) return NULL;
  if (A0->level < 1) { *err = -2; oc_ct_free(A0); return NULL; }
  int lvl = A0->level;
  double *vec = (double *)malloc(sizeof(double) * n2sq);
  i64 *m = (i64 *)malloc(sizeof(i64) * N);
  oc_ct **Ak = (oc_ct **)calloc(n, sizeof(oc_ct *));
  oc_ct *Bb = oc_ct_copy(c, A0), *Bpb = oc_rotate(c, A0, -(i64)n);
  for (int b = 0; b * n1z < n && Bb && Bpb; b++) {
    if (b > 0) {
      oc_ct *t = oc_rotate(c, Bb, n1z); oc_ct_free(Bb); Bb = t;
      t = oc_rotate(c, Bpb, n1z); oc_ct_free(Bpb); Bpb = t;
      if (!Bb || !Bpb) break;
    }
    u64 *d1 = oc_decompose(c, poly(c, Bb, 1, 0), lvl);
    u64 *d2 = oc_decompose(c, poly(c, Bpb, 1, 0), lvl);
    for (int r = 0; r < n1z && b * n1z + r < n; r++) {
      int k = b * n1z + r;
      u64 g = oc_galois_of_step(c, r);
      /* masks encoded at scale q_lvl: the rescale restores Bb's scale */
      double ql = (double)c->mods[lvl];
      oc_ct *acc = ct_new(c, lvl, 1, Bb->scale * ql);
      oc_ct *h = hoisted_rot(c, Bb, d1, g, err);
      col_mask(n, k, 0, vec);
      pt_int(c, vec, n2sq, ql, m);
      qp_pmult_acc(c, acc, h, m);
      oc_ct_free(h);
      if (k > 0) {
        h = hoisted_rot(c, Bpb, d2, g, err);
        col_mask(n, k, 1, vec);
        pt_int(c, vec, n2sq, ql, m);
        qp_pmult_acc(c, acc, h, m);
        oc_ct_free(h);
      }
      if (fused) {
        Ak[k] = oc_moddown_rescale(c, acc);
      } else {
        oc_ct *md = oc_moddown(c, acc);
        Ak[k] = oc_rescale(c, md);
        oc_ct_free(md);
      }
      if (Ak[k]) Ak[k]->scale = Bb->scale;
      oc_ct_free(acc);
    }
    free(d1); free(d2);
  }
  oc_ct_free(Bb); oc_ct_free(Bpb); oc_ct_free(A0);
  free(vec); free(m);
  for (int k = 0; k < n; k++)
    if (!Ak[k]) { if (!*err) *err = -4; for (int j = 0; j < n; j++) oc_ct_free(Ak[j]); free(Ak); return NULL; }
  return Ak;
}

/* B side: B_k = R^k T b.  C_0 = T b, C_b = Rot(C_{b-1}, n n1t),
 * B_k = ModDown(HR(C_b, n r)) for k = b n1t + r (C_b itself for r = 0). */
static oc_ct **side_b(const oc_ctx *c, const oc_ct *cb, int n, int n1t, int npt, int *err) {
  oc_ct *Cb = tau_dcd(c, cb, n, n1t, npt, err);
  if (!Cb) return NULL;
  int lvl = Cb->level;
  oc_ct **Bk = (oc_ct **)calloc(n, sizeof(oc_ct *));
  for (int b = 0; b * n1t < n && Cb; b++) {
    if (b > 0) {
      oc_ct *t = oc_rotate(c, Cb, (i64)n * n1t); oc_ct_free(Cb); Cb = t;
      if (!Cb) break;
    }
    u64 *d1 = oc_decompose(c, poly(c, Cb, 1, 0), lvl);
    for (int r = 0; r < n1t && b * n1t + r < n; r++) {
      int k = b * n1t + r;
      if (r == 0) Bk[k] = oc_ct_copy(c, Cb);
      else {
        oc_ct *h = hoisted_rot(c, Cb, d1, oc_galois_of_step(c, (i64)n * r), err);
        if (h) Bk[k] = oc_moddown(c, h);
        oc_ct_free(h);
      }
    }
    free(d1);
  }
  oc_ct_free(Cb);
  for (int k = 0; k < n; k++)
    if (!Bk[k]) { if (!*err) *err = -4; for (int j = 0; j < n; j++) oc_ct_free(Bk[j]); free(Bk); return NULL; }
  return Bk;
}

/* both sides dropped to their common (lowest) level */
static void align_sides(const oc_ctx *c, oc_ct **Ak, oc_ct **Bk, int n) {
  int lv = Ak[0]->level < Bk[0]->level ? Ak[0]->level : Bk[0]->level;
  for (int k = 0; k < n; k++) {
    if (Ak[k]->level > lv) { oc_ct *t = oc_drop(c, Ak[k], lv); oc_ct_free(Ak[k]); Ak[k] = t; }
    if (Bk[k]->level > lv) { oc_ct *t = oc_drop(c, Bk[k], lv); oc_ct_free(Bk[k]); Bk[k] = t; }
  }
}

/* acc += sum_k Relin(Tensor(A_k, B_k)) */
static oc_ct *accumulate(const oc_ctx *c, oc_ct *acc, oc_ct **Ak, oc_ct **Bk, int n) {
  for (int k = 0; k < n; k++) {
    oc_ct *p = oc_mult(c, Ak[k], Bk[k]);
    if (!acc) acc = p;
    else { add_into(c, acc, p); oc_ct_free(p); }
  }
  return acc;
}

/* Lazy relinearisation (a variant, not the paper's order): the tensors of
 * all products are summed in three components and relinearised once.
 * acc3 = u64[3][l+1][N] running sum (NULL: start a new one). */
static u64 *accumulate_tensors(const oc_ctx *c, u64 *acc3, oc_ct **Ak, oc_ct **Bk, int n) {
  int nq = Ak[0]->nlimbs;
  size_t words = (size_t)3 * nq * c->N;
  u64 *t3 = alloc_u64(words);
  if (!acc3) acc3 = alloc_u64(words);  /* zeroed */
  for (int k = 0; k < n; k++) {
    oc_tensor(c, Ak[k], Bk[k], t3);
    for (int p = 0; p < 3; p++)
      for (int l = 0; l < nq; l++) {
        u64 q = c->mods[l];
        u64 *a = acc3 + ((size_t)p * nq + l) * c->N, *t = t3 + ((size_t)p * nq + l) * c->N;
        for (u64 i = 0; i < c->N; i++) a[i] = addmod(a[i], t[i], q);
      }
  }
  free(t3);
  return acc3;
}

static void free_list(oc_ct **l, int n) {
  if (!l) return;
  for (int k = 0; k < n; k++) oc_ct_free(l[k]);
  free(l);
}

/* Permutation of the folded A side: C^k applied after Z, output (i, j) takes
 * A_{i, (i + j + k) mod n} (phi^k(sigma(A)) of Eq. 5 read as one map). */
static int *perm_phi_sigma(int n, int k) {
  int *p = (int *)malloc(sizeof(int) * n * n);
  for (int i = 0; i < n; i++)
    for (int j = 0; j < n; j++) p[i * n + j] = i * n + (i + j + k) % n;
  return p;
}
void oc_perm_phi_sigma(int n, int k, int *out) {
  int *p = perm_phi_sigma(n, k);
  memcpy(out, p, sizeof(int) * n * n);
  free(p);
}

/* A side with the masks of C^k folded into Z (section 4.1.1 computes
 * C^k(Z a) with two masks and a level of its own): phi^k o sigma is a
 * permutation whose diagonals are C^k's masks times Z's diagonals, with
 * Z's diagonal indices (in (-n, n)), so A_k = U_k a is one double-hoisted
 * BSGS transform on a with Z's geometry and keys, one level in all. */
static oc_ct **side_a_folded(const oc_ctx *c, const oc_ct *ca, int n, int n1z, int *err) {
  oc_ct **Ak = (oc_ct **)calloc(n, sizeof(oc_ct *));
  int n2 = ceil_div(n, n1z);
  for (int k = 0; k < n; k++) {
    int *p = perm_phi_sigma(n, k);
    lt_perm U = {n * n, p, NULL};
    Ak[k] = lintrans(c, ca, &U, 1, n1z, -n2, n2, 0, err);
    free(p);
    if (!Ak[k]) {
      if (!*err) *err = -4;
      for (int j = 0; j < n; j++) oc_ct_free(Ak[j]);
      free(Ak);
      return NULL;
    }
  }
  return Ak;
}

/* flags: 1 = lazy relinearisation (the n tensors summed, relinearised once),
 * 2 = ModDown and Rescale of the A side as one rounding; both variants of
 * the paper's order.  4 = the A side with the masks folded into Z
 * (side_a_folded): two levels in all instead of three (no decomposition of
 * Z, not with flag 2). */
oc_ct *oc_matmul_lazy(const oc_ctx *c, const oc_ct *ca, const oc_ct *cb, int n, int n1z, int n1t, int npz,
                      int npt, int flags, int *err) {
  const int lazy = flags & 1, folded = flags & 4;
  *err = 0;
  if (ca->qp || cb->qp || ca->level != cb->level) { *err = -2; return NULL; }
  if ((u64)n * n > c->N / 2 || n % n1z || n % n1t || npz < 1 || npt < 1) { *err = -1; return NULL; }
  if (folded && ((flags & 2) || npz < n - 1)) { *err = -1; return NULL; }
  oc_ct **Ak = folded ? side_a_folded(c, ca, n, n1z, err) : side_a(c, ca, n, n1z, npz, flags & 2, err);
  if (!Ak) return NULL;
  oc_ct **Bk = side_b(c, cb, n, n1t, npt, err);
  if (!Bk) { free_list(Ak, n); return NULL; }
  align_sides(c, Ak, Bk, n);
  if (Ak[0]->level < 1) { *err = -2; free_list(Ak, n); free_list(Bk, n); return NULL; }
  oc_ct *acc;
  if (lazy) {
    u64 *acc3 = accumulate_tensors(c, NULL, Ak, Bk, n);
    acc = oc_relin(c, acc3, Ak[0]->level, Ak[0]->scale * Bk[0]->scale);
    free(acc3);
  } else {
    acc = accumulate(c, NULL, Ak, Bk, n);
  }
  oc_ct *out = oc_rescale(c, acc);
  oc_ct_free(acc);
  free_list(Ak, n); free_list(Bk, n);
  return out;
}

oc_ct *oc_matmul_ex(const oc_ctx *c, const oc_ct *ca, const oc_ct *cb, int n, int n1z, int n1t, int npz, int npt,
                    int *err) {
  return oc_matmul_lazy(c, ca, cb, n, n1z, n1t, npz, npt, 0, err);
}

oc_ct *oc_matmul(const oc_ctx *c, const oc_ct *ca, const oc_ct *cb, int n, int n1z, int n1t, int *err) {
  return oc_matmul_ex(c, ca, cb, n, n1z, n1t, n - 1, n - 1, err);
}

/* ------------------------------------------------------------------------ */
/* Covariance of a centred dataset (Algorithm HCovMtrx, section 5.2).        */
/* x[r k + j] = block (row block r, feature block j).  Block (a, b) of        */
/* X^T X / s for b <= a is Rescale(sum_r sum_k Relin(Tensor(A_k, B_k))) with */
/* A from G(x[r k + a]) scaled by 1/s and B from x[r k + b]; blocks a < b    */
/* are G of block (b, a); every block ends at one level.                     */
/* ------------------------------------------------------------------------ */
int oc_covariance_lazy(const oc_ctx *c, oc_ct *const *x, int rb, int k, int n, u64 n_samples, int n1z, int n1t,
                       int npz, int npt, int n1g, int flags, oc_ct **out) {
  int err = 0;
  const int lazy = flags & 1;
  int level = x[0]->level;
  oc_ct **acc = (oc_ct **)calloc(k * k, sizeof(oc_ct *));
  u64 **acc3 = (u64 **)calloc(k * k, sizeof(u64 *));
  int acc_level = 0;
  double acc_scale = 0;
  for (int r = 0; r < rb; r++) {
    oc_ct ***A = (oc_ct ***)calloc(k, sizeof(oc_ct **)), ***B = (oc_ct ***)calloc(k, sizeof(oc_ct **));
    for (int a = 0; a < k; a++) {
      oc_ct *xt = oc_lt_transpose(c, x[r * k + a], n, n1g, 1.0 / (double)n_samples, &err);
      if (!xt) return err ? err : -1;
      A[a] = side_a(c, xt, n, n1z, npz, flags & 2, &err);
      oc_ct_free(xt);
      if (!A[a]) return err ? err : -1;
    }
    for (int b = 0; b < k; b++) {
      oc_ct *xb = oc_drop(c, x[r * k + b], level - 1);
      B[b] = side_b(c, xb, n, n1t, npt, &err);
      oc_ct_free(xb);
      if (!B[b]) return err ? err : -1;
    }
    for (int a = 0; a < k; a++) align_sides(c, A[a], B[0], n);
    for (int b = 0; b < k; b++) align_sides(c, A[0], B[b], n);
    acc_level = A[0][0]->level;
    acc_scale = A[0][0]->scale * B[0][0]->scale;
    for (int a = 0; a < k; a++)
      for (int b = 0; b <= a; b++) {
        if (lazy) acc3[a * k + b] = accumulate_tensors(c, acc3[a * k + b], A[a], B[b], n);
        else acc[a * k + b] = accumulate(c, acc[a * k + b], A[a], B[b], n);
      }
    for (int a = 0; a < k; a++) free_list(A[a], n);
    for (int b = 0; b < k; b++) free_list(B[b], n);
    free(A); free(B);
  }
  for (int a = 0; a < k; a++)
    for (int b = 0; b <= a; b++) {
      if (lazy) {
        acc[a * k + b] = oc_relin(c, acc3[a * k + b], acc_level, acc_scale);
        free(acc3[a * k + b]);
      }
      out[a * k + b] = oc_rescale(c, acc[a * k + b]);
      oc_ct_free(acc[a * k + b]);
    }
  free(acc);
  free(acc3);
  for (int a = 0; a < k; a++)
    for (int b = a + 1; b < k; b++) {
      out[a * k + b] = oc_lt_transpose(c, out[b * k + a], n, n1g, 1.0, &err);
      if (!out[a * k + b]) return err ? err : -1;
    }
  if (k > 1) {
    int fl = out[1]->level;
    for (int a = 0; a < k; a++)
      for (int b = 0; b <= a; b++) {
        oc_ct *t = oc_drop(c, out[a * k + b], fl);
        oc_ct_free(out[a * k + b]);
        out[a * k + b] = t;
      }
  }
  return 0;
}

int oc_covariance(const oc_ctx *c, oc_ct *const *x, int rb, int k, int n, u64 n_samples, int n1z, int n1t, int npz,
                  int npt, int n1g, oc_ct **out) {
  return oc_covariance_lazy(c, x, rb, k, n, n_samples, n1z, n1t, npz, npt, n1g, 0, out);
}
