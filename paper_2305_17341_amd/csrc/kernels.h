// Launch wrappers for the gfx950 kernels (internal).
#pragma once
#include <functional>

#include "he_internal.h"

// Limb batch -> modulus index map; -1 skips the limb.
struct LimbMap {
  int n;                 // period
  short idx[960];
  // the transforms (launch_ntt) only: with slot_per > 0, limb k lives in
  // memory slot (k / slot_per) * slot_stride + slot_off + k % slot_per (for
  // example the special-prime limbs of an R_{Q_l P} element, in place)
  short slot_per = 0, slot_stride = 0, slot_off = 0;
};

struct DeviceTables {
  int logN = 0;
  u64 N = 0;
  int nmods = 0;
  ModConst* mc = nullptr;      // [nmods]
  int bits[HE_MAXMOD] = {};    // host copy: bit length of each modulus
  u64* psi = nullptr;          // [nmods][N] psi^brv(k)
  u64* psi_sh = nullptr;
  u64* ipsi = nullptr;         // [nmods][N] psi^-brv(k)
  u64* ipsi_sh = nullptr;
  double* psi_f = nullptr;     // psi^brv as doubles (exact, used for moduli below 2^50)
  double* ipsi_f = nullptr;
  // double-double FFT tables for the canonical embedding
  double* fft_tw = nullptr;    // [N/2][4] exp(-2 pi i k / N) as (re_hi, re_lo, im_hi, im_lo)
  double* zeta = nullptr;      // [N][4] (cos(pi i/N), sin(pi i/N)) dd
  u32* rotgroup = nullptr;     // [N/2] 5^j mod 2N
  u64* cdt = nullptr;          // [38] Gaussian inversion table
};

// transforms
void launch_ntt(const DeviceTables& T, u64* data, int nlimbs, const LimbMap& map, bool inverse, hipStream_t s);
// Inverse NTT of src into data (same layout) with limb k's result times
// scales[2 m] (Shoup pairs by modulus m) in place of N^-1; false (nothing
// launched) without the register-blocked NTT
bool launch_intt_scaled(const DeviceTables& T, u64* data, const u64* src, int nlimbs, const LimbMap& map,
                        const u64* scales, hipStream_t s);
// forward NTT of npoly x nq limbs y, then out = (x - y) c mod q_t with x
// [npoly][x_stride][N] and c pairs (value, Shoup companion) per t < nq
void launch_ntt_fwd_sub(const DeviceTables& T, u64* y, int nq, int npoly, const LimbMap& map, const u64* x,
                        int x_stride, const u64* cpairs, u64* out, hipStream_t s);

// Decompose's conversion fused into the forward NTT of the digits (false:
// not available for this ring size; nothing was launched)
struct FbcTable;
// generic-path digits ([0, q) residues) into the key inner products' operand
// form: limbs of moduli below 2^46 as centred doubles (bit patterns)
void launch_digits_f64(const DeviceTables& T, u64* d, int nlimbs, const LimbMap& map, hipStream_t s);
bool launch_modup_ntt(const DeviceTables& T, u64* digits, const u64* y, const u64* ntt_in, int level, int L,
                      int alpha, int beta, const FbcTable* tabs, int batch, const LimbMap& rows_map, hipStream_t s);

// data movement / elementwise (data laid out [nlimbs][N], limb k uses map)
void launch_automorph(const DeviceTables& T, u64* out, const u64* in, int nlimbs, u64 g, hipStream_t s);
void launch_add(const DeviceTables& T, u64* out, const u64* a, const u64* b, int nlimbs, const LimbMap& m, hipStream_t s);
void launch_sub(const DeviceTables& T, u64* out, const u64* a, const u64* b, int nlimbs, const LimbMap& m, hipStream_t s);
void launch_mul(const DeviceTables& T, u64* out, const u64* a, const u64* b, int nlimbs, const LimbMap& m, hipStream_t s);
// out = a * b where b has period b_limbs (b limb = k % b_limbs)
void launch_mul_bcast(const DeviceTables& T, u64* out, const u64* a, const u64* b, int nlimbs, int b_limbs,
                      const LimbMap& m, hipStream_t s);
// acc += a * b (b broadcast with period b_limbs)
void launch_mul_acc(const DeviceTables& T, u64* acc, const u64* a, const u64* b, int nlimbs, int b_limbs,
                    const LimbMap& m, hipStream_t s);
// out (+)= sum_t a[t] * p[t] (p[t] broadcast with period b_limbs), nterms pairs
#define SUM_MAX_TERMS 64  // at most 64 signed products below q < 2^46: sums below 2^52
void launch_mul_sum(const DeviceTables& T, u64* out, const u64* const* a, const u64* const* p, int nterms,
                    int nlimbs, int b_limbs, const LimbMap& m, bool accumulate, hipStream_t s);
// outs[g] = sum_t a[t] * p[g * nterms + t] for g < nouts (null p: term absent);
// false (nothing launched) beyond SUM_MAX_OUTS outputs or SUM_MAX_TERMS terms
#define SUM_MAX_OUTS 4
bool launch_mul_sum_multi(const DeviceTables& T, u64* const* outs, int nouts, const u64* const* a,
                          const u64* const* p, int nterms, int nlimbs, int b_limbs, const LimbMap& m,
                          hipStream_t s);
// out = a * c_k for a per-limb constant (host array, Shoup)
void launch_mul_const(const DeviceTables& T, u64* out, const u64* a, int nlimbs, const u64* consts /*[map.n]*/,
                      const LimbMap& m, hipStream_t s);
void launch_neg(const DeviceTables& T, u64* out, const u64* a, int nlimbs, const LimbMap& m, hipStream_t s);
// batch pairs of ciphertexts [2][batch][nl] -> [3][batch][nl] (accumulate: added onto out3)
// sum of npairs tensors (a[p], b[p] over Q_l, [2][B][nl] each) into the
// three-component [3][B][nl] out3, or added onto it; a_packed[p] (b_packed)
// set: a[p]'s limbs of FP64 moduli are stored packed (the fused ModDown's
// pack_out layout)
void launch_tensor_sum(const DeviceTables& T, u64* out3, const u64* const* a, const u64* const* b, int npairs, int nl,
                       int batch, bool accumulate, hipStream_t s, const bool* a_packed = nullptr,
                       const bool* b_packed = nullptr);
void launch_tensor(const DeviceTables& T, u64* out3, const u64* a, const u64* b, int nl, int batch, bool accumulate,
                   hipStream_t s);
void launch_int_to_limbs(const DeviceTables& T, u64* out, const i64* in, int nlimbs, const LimbMap& m, hipStream_t s);

// key switching pieces
struct FbcTable {
  // source set S (ns primes) -> any target modulus:
  // y_a = x_a * hatinv_a mod q_a ; out_t = sum_a y_a * hat_{a,t} mod t
  int ns = 0;
  int src[8];
  u64 hatinv[8], hatinv_sh[8];
  u64* hat_t = nullptr;     // device [ns][nmods] (hat_a mod t)
  u64* hat_t_sh = nullptr;  // device [ns][nmods]
  // exact centred lift (ModDown): D = prod of the sources as 4 words, its
  // cofactors D / q_a, the sources as doubles, and D mod t (Shoup pairs)
  u64 Dw[4] = {0, 0, 0, 0};
  u64 Hw[8][4];
  double qd[8];
  u64* D_mod_t = nullptr;   // device [nmods][2]
  double* hat_f = nullptr;  // device [ns][nmods][3]: hat mod t, 2^32 hat mod t, D mod t (FP64 path)
  // The lift as a dot product of 7-bit digits (ModDown tables only): the
  // record of a coefficient holds digit i of source value a at byte 9 a + i
  // and the quotient at byte 9 ns, in kw words; cdig [nmods][8][kw] holds,
  // for target t and row j < 7, digit j of the constant of each record byte:
  // hat_(a,t) 2^(7 i) mod q_t, and -D mod q_t for the quotient.
  u64* cdig = nullptr;
  int kw = 0;
};
// digits[j][pos] (pos over Q_l then P): own limbs copy ntt_in, others are the
// coefficient-domain conversion of digit j (to be transformed by the caller)
void launch_modup(const DeviceTables& T, u64* digits, const u64* coef, const u64* ntt_in, int level, int L,
                  int alpha, int beta, const FbcTable* tabs /* host array [beta] */, int batch, hipStream_t s);
// ModDown's conversion fused into the forward NTT of the Q limbs (the tail
// (x - y) P^-1 in its block pass): scratch y [npoly][nq][N] and V
// [npoly][ns + 1][N]; false when the ring size has no register-blocked NTT
// Inverse NTT, in place, of the same limbs of many R_{Q_l P} elements (the
// ModDown sources of a set of hoisted rotations): in element e (bases[e]),
// limb j < per_elem lives at slot (j / per) * stride + off + j % per; map
// gives the modulus of limb j by j % map.n (map.n = per).  One launch per 64
// elements.
// With rec_tab and rec: the sources are those of the ModDown table rec_tab
// (per = its ns) and the last pass writes their digit records to rec
// ([element][per_elem / per][per + 1][N]) instead of the limbs.
void launch_intt_many(const DeviceTables& T, const std::vector<u64*>& bases, int per_elem, int per, int stride,
                      int off, const LimbMap& map, hipStream_t s, const FbcTable* rec_tab = nullptr,
                      u64* rec = nullptr);
// xp_coef: the source limbs in the coefficient domain, [npoly][ns][N]; or,
// with src_stride > 0, limb a of poly p at slot p * src_stride + src_off + a
// (the sources transformed in place inside the R_{Q_l P} element)
// whether a fused ModDown into nq target limbs with this table takes digit
// records (the int8 lift); only then may V arrive filled (v_ready)
bool fbc_digit_path(const DeviceTables& T, const FbcTable& tab, int nq);
// pack_out: out's limbs of FP64 moduli (at most 46 bits) are stored packed in
// their N-word slots: the low 32 bits of every residue, then one high byte
// each (moduli of at most 40 bits) or two
bool launch_moddown_fused(const DeviceTables& T, const u64* xp_coef, int nq, int npoly, const FbcTable& tab,
                          const u64* x, int x_stride, const u64* pinv, u64* out, u64* y, u64* V, hipStream_t s,
                          int src_stride = 0, int src_off = 0, bool v_ready = false, bool pack_out = false);
// y[npoly][nq] = exact centred lift of the source limbs xp[npoly][ns] to each q_t
void launch_fbc_to_q(const DeviceTables& T, u64* y, const u64* xp_coef, int nq, int npoly, const FbcTable& tab,
                     hipStream_t s);
void launch_moddown_final(const DeviceTables& T, u64* out, const u64* x, const u64* y, int nq,
                          const u64* pinv /*device [nmods] Shoup pairs*/, int npoly, int x_stride_limbs,
                          hipStream_t s);
// hoisted rotation: out[2][nqp][N] = sum_j pi_g(d_j) * key_j (+ P pi_g(c0) on Q limbs)
void launch_multsum(const DeviceTables& T, u64* out, const u64* digits, const u64* key, const u64* c0,
                    const u64* pmod /*device [nmods][2]*/, int level, int L, int alpha, int beta, u64 g,
                    int batch, hipStream_t s);
// nrot hoisted rotations of the same digits (Galois elements gs[], keys[]) into
// outs[r] (each [2][batch][nqp][N]); digits read from HBM once per launch.
// With masks (plaintexts [nqp][N] in R_{Q_l P}, one per rotation) the outputs
// are mask (.) rotation, added onto outs[r] when `accumulate`.
#define MR_MAX 64
// A second stream forked from and joined to the launching stream with
// events (default priority).  With it, a multi-rotation launch runs the
// kernel of its 60-bit limbs there, beside the kernel of its FP64 limbs: the
// one is bound by integer and FP64 issue, the other mostly by HBM.
struct ForkStream {
  hipStream_t aux = nullptr;
  hipEvent_t fork = nullptr, join = nullptr;
};
void launch_multsum_rot(const DeviceTables& T, u64* const* outs, const u64* const* keys, const u64* gs, int nrot,
                        const u64* digits, const u64* c0, const u64* pmod, int level, int L, int alpha, int beta,
                        int batch, hipStream_t s, const u64* const* masks = nullptr, bool accumulate = false,
                        const ForkStream* fs = nullptr);
// two bases under the same keys: outs[r] = masks[r] * rotation r of base 1
// (digits, c0) + masks2[r] * rotation r of base 2 (digits2, c02), each key
// word loaded once; false (nothing launched) where that does not apply
bool launch_multsum_rot_pair(const DeviceTables& T, u64* const* outs, const u64* const* keys, const u64* gs, int nrot,
                             const u64* digits, const u64* c0, const u64* const* masks, const u64* digits2,
                             const u64* c02, const u64* const* masks2, const u64* pmod, int level, int L, int alpha,
                             int beta, int batch, hipStream_t s);
// Key inner products handed to a sink instead of being launched (merged
// launches of several products): the arguments of one launch_multsum_rot or
// launch_multsum call
struct KsWork {
  std::vector<u64*> outs;
  std::vector<const u64*> keys;
  std::vector<u64> gs;
  std::vector<const u64*> masks;  // empty: plain outputs
  bool accumulate = false;
  const u64* digits = nullptr;
  const u64* c0 = nullptr;
  const u64* pmod = nullptr;
  int level = 0, beta = 0, B = 1;
};
using KsSink = std::function<void(KsWork&&)>;
// set the calling thread's sink (null: launch as usual); returns the previous one
KsSink* ks_sink_exchange(KsSink* s);
// one launch per member count over every item of `works` (any levels): the
// same residues as their own launch_multsum_rot calls.  `table` is device
// memory of multsum_list_table_bytes() bytes for the work table (uploaded
// from pageable memory: not for use under stream capture).
size_t multsum_list_table_bytes(const DeviceTables& T, const std::vector<KsWork>& works, int L, int alpha);
void launch_multsum_list(const DeviceTables& T, const std::vector<KsWork>& works, void* table, size_t table_bytes,
                         int L, int alpha, hipStream_t s);
// P-lift: out[2][nqp][N] = (P c0, P c1) on Q limbs, 0 on P limbs
void launch_plift(const DeviceTables& T, u64* out, const u64* c, const u64* pmod, int level, int alpha, int npoly,
                  hipStream_t s);
// rescale pieces
void launch_rescale_lift(const DeviceTables& T, u64* t, const u64* top_coef, int l, int nout, int npoly,
                         hipStream_t s);
// Rescale's lift fused into the forward NTT of the kept limbs and its tail
// (x - t) q_l^-1 into the block pass: t scratch [npoly][nout][N], top_coef
// the top limbs in the coefficient domain; false when the ring size has no
// register-blocked NTT
bool launch_rescale_fused(const DeviceTables& T, u64* t, const u64* top_coef, int l, int nout, int npoly,
                          const u64* x, int x_stride, const u64* cpairs, u64* out, hipStream_t s);
void launch_rescale_final(const DeviceTables& T, u64* out, const u64* x, const u64* t, int l, int npoly,
                          int x_stride_limbs, const u64* qlinv /*device [l][2]*/, hipStream_t s);

// randomness (Philox4x64-10, counter = (coefficient, c1, c2, c3), key = (seed, tag))
void launch_sample_uniform(const DeviceTables& T, u64* out, int nlimbs, const LimbMap& m, u64 seed, u64 tag,
                           u64 c2, u64 c3, hipStream_t s);
void launch_sample_ternary(const DeviceTables& T, i64* out, u64 seed, u64 tag, u64 c1, u64 c2, u64 c3,
                           hipStream_t s);
void launch_sample_gauss(const DeviceTables& T, i64* out, u64 seed, u64 tag, u64 c1, u64 c2, u64 c3,
                         hipStream_t s);
void launch_add_int(i64* out, const i64* a, const i64* b, u64 N, hipStream_t s);
// m <- round(m * mant / 2^shift) (halves away from zero), 1 <= shift < 128, |m| mant < 2^127
void launch_scale_int(i64* m, u64 mant, int shift, u64 N, hipStream_t s);
// switching key b part: b = e - a s (+ pmod s' on the digit's primes)
void launch_swk_b(const DeviceTables& T, u64* b, const u64* a, const u64* e, const u64* s_ntt, const u64* sp_ntt,
                  const u64* pmod, int nlimbs_total, int digit, int alpha, int L, hipStream_t s);
// the FP64 limbs (at most F64_LAZY_BITS bits) of a switching key of nblocks
// blocks of nmods limbs rewritten in place as doubles, the form the key inner
// products read
void launch_key_f64(const DeviceTables& T, u64* key, int nblocks, int nmods, hipStream_t s);

// canonical embedding (double-double FFT)
void launch_encode(const DeviceTables& T, i64* out, const double* z, int nz, int batch, double delta, void* scratch,
                   hipStream_t s);
size_t encode_scratch_bytes(const DeviceTables& T, int batch);
void launch_decode(const DeviceTables& T, double* out, const i64* m, int batch, const double* inv_scale,
                   void* scratch, hipStream_t s);
// decryption helpers
void launch_centre_to_int(const DeviceTables& T, i64* out, const u64* coef, int mod, hipStream_t s);

// launch-shape knobs: "ms_members", "mr_members", "mr_rotations", "ntt_interleave",
// "ew_interleave", "cov_row_blocks" (false: unknown name or value)
bool knob_set(const char* name, int value);
bool knob_get(const char* name, int* value);

// algorithmic modular products, split by arithmetic (f: lazy FP64 for moduli
// below 2^46, i: 64-bit integer)
struct Mm {
  double f = 0, i = 0;
  void add(int bits, double n) { (bits <= F64_LAZY_BITS ? f : i) += n; }
};
Mm mm_map(const DeviceTables& T, const LimbMap& m, int nlimbs, double per_limb);

// device-to-device copies, timed under `family` while profiling is on
hipError_t copy_async(const char* family, void* dst, const void* src, size_t bytes, hipStream_t s);
hipError_t copy2d_async(const char* family, void* dst, size_t dpitch, const void* src, size_t spitch, size_t width,
                        size_t height, hipStream_t s);

// per-family device timing (HIP events around launches)
void prof_enable(bool on);
bool prof_enabled();
bool prof_read(const char* family, double* ms, u64* launches, double* bytes);
bool prof_read_ops(const char* family, double* mm_f64, double* mm_int, double* unit_bytes);
std::vector<std::string> prof_families();
