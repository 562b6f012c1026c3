// Host runtime declarations (internal).
#pragma once
#include <functional>
#include <list>
#include <memory>
#include <mutex>
#include <set>
#include <string>
#include <vector>

#include "../../include/he_mi355x.h"
#include "kernels.h"

struct HeError {
  he_status st;
  std::string msg;
};
[[noreturn]] inline void fail(he_status st, const std::string& m) { throw HeError{st, m}; }
void hip_check(hipError_t e, const char* what);
extern thread_local std::string g_last_error;
u64 shoup_pre(u64 w, u64 q);

// randomness stream tags (Philox key = (seed, tag))
enum { TAG_SK = 1, TAG_PK_A = 2, TAG_PK_E = 3, TAG_SWK_A = 4, TAG_SWK_E = 5, TAG_ENC_V = 6, TAG_ENC_E0 = 7,
       TAG_ENC_E1 = 8 };

enum { LT_SIGMA = 0, LT_TAU = 1, LT_TRANSPOSE = 2 };

// BSGS geometry: indices a (n1 i + j), j in [0, n1), i in [i_lo, i_hi)
struct LtGeom {
  int a, n1, i_lo, i_hi;
};
LtGeom lt_geom(int kind, int n, int n1);
std::vector<int> make_perm(int kind, int n);
int default_n1(int n);

// diagonal convergence decomposition
enum { DCD_Z1 = 0, DCD_Z2 = 1, DCD_T = 2 };
struct DcdFactor {
  std::vector<int> perm;  // output t takes input perm[t]; -1 = zero row
  LtGeom G;
};
std::vector<DcdFactor> dcd_chain(int n, const std::vector<int>& perm, int which, int nprime, int n1);
void bsgs_steps(const std::vector<int>& perm, const LtGeom& G, std::set<long>& out, int n1p = 0);
void lintrans_steps(int kind, int n, int n1, int nprime, std::set<long>& s);
std::vector<long> matmul_steps(int n, int n1z, int n1t, int npz, int npt, bool folded = false);
std::vector<long> transpose_steps(int n, int n1);

// the moduli (Q then P) and their NTT roots psi for these prime sizes (host only)
void params_moduli(int logN, const std::vector<int>& bits, u64* moduli, u64* psi);
// measured rate of one kind of modular product (microbench.hip)
void modmul_peak(int kind, u64 iters, int blocks, double* rate, double* ms);

// replaces a ciphertext that ran out of levels by a fresh one (client side)
using RefreshFn = std::function<void(HeCt&)>;

// A batched product recorded as a HIP graph: replays run the whole launch
// sequence with one call.  The graph's temporaries and outputs live in its
// own arena, which nothing else allocates from.
struct MmGraph {
  std::vector<u64> key;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  std::unique_ptr<DevPool> arena;
  std::vector<HeCt> outs;
  MmGraph() = default;
  MmGraph(const MmGraph&) = delete;
  MmGraph& operator=(const MmGraph&) = delete;
  // The owner synchronises the stream a replay ran on before destroying a
  // recording (HIP leaves destroying an executable graph that is still
  // running undefined); the device-wide wait here covers any other path.
  ~MmGraph() {
    if (exec) (void)hipDeviceSynchronize();
    outs.clear();
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
  }
};

// A block covariance accumulated over calls (Algorithm HCovMtrx): the
// product options, the level the dataset blocks share, and the k^2 running
// sums of XtX over the row blocks seen (three-component tensor sums with lazy
// relinearisation, else relinearised products).
struct CovState {
  int k = 0, n = 0;
  u64 n_samples = 0;
  int n1z = 0, n1t = 0, n1g = 0, npz = 0, npt = 0;
  bool lazy = false, fused = false;
  int level = -1;
  long row_blocks = 0;
  int acc_level = 0;
  double acc_scale = 0;
  std::vector<HeCt> acc;
  std::vector<DevBuf> acc3;
  std::vector<bool> set;
};

struct HeCtxImpl {
  int logN = 0;
  u64 N = 0;
  int L = 0, alpha = 0, beta = 0, nmods = 0;
  // log N 12..16: the conversions of Decompose, ModDown and Rescale are fused
  // into the forward NTT passes (register-blocked NTT available)
  bool fused_conv = false;
  u64 mods[HE_MAXMOD];
  double delta = 0, sigma = 0;
  u64 seed = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  // second stream of the multi-rotation launches (see ForkStream)
  ForkStream fork;
  // device the context was created on, and that device's copy of the
  // allocation-free entry points' workspace
  int device = 0;
  void* noalloc_ws = nullptr;
  DevPool pool;
  DeviceTables T;
  std::vector<ModConst> mc;
  std::vector<DevBuf> tables;
  std::vector<std::vector<FbcTable>> up;  // [level][digit]
  std::vector<FbcTable> down_rs;          // [level]: sources q_l and P (empty when alpha > 3)
  FbcTable down;                          // P -> Q
  DevBuf pmod, pinv, qlinv;
  DevBuf pqlinv;  // [level][nmods][2]: (P q_l)^-1 mod q_k with Shoup companions
  DevBuf up_scale;  // [level][nmods][2]: N^-1 hatinv_t mod q_t (Decompose's digit sources)
  DevBuf s_ntt, pk;
  bool have_sk = false;
  std::map<u64, DevBuf> keys;             // Galois element -> key; 0 = relinearisation (FP64 limbs as doubles)
  std::map<std::string, DevBuf> ptcache;
  // a transform's diagonals present (giant, baby step) and their plaintexts
  // (entries of ptcache, kept for the context's life)
  struct LtPlan {
    std::vector<std::pair<int, int>> ij;
    std::vector<const u64*> pts;
  };
  std::map<std::string, LtPlan> ltplans;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  double last_ms = 0;
  long n_decompose = 0, n_multsum = 0, n_moddown = 0;
  std::list<MmGraph> graphs;  // most recently used first (declared after the pool: destroyed before it)

  ~HeCtxImpl();
  void init(const he_params* p, const he_device* dev, u64 seed);

  int nq_of(int level) const { return level + 1; }
  int nqp_of(int level) const { return level + 1 + alpha; }
  int beta_at(int level) const { return (level + alpha) / alpha; }
  int qp_mod(int level, int pos) const { return pos <= level ? pos : L + 1 + (pos - level - 1); }
  LimbMap qmap(int nq) const;
  LimbMap qpmap(int level) const;
  LimbMap one(int mod) const;
  u64 galois(long step) const;
  u64* table_upload(const void* host, size_t bytes);

  HeCt ct_new(int level, bool qp, double scale, int B = 1);
  HeCt ct_copy(const HeCt& x);
  void copy_limbs(u64* dst, const u64* src, size_t nlimbs, const char* family = "copy_limbs");

  DevBuf encode_batch(const double* z_host, int nz, int batch, double delta);
  void int_to_ntt(u64* out, const i64* m, const LimbMap& map);

  void keygen_secret();
  void swk_gen(const u64* sp, u64 kid, DevBuf& out);
  void keygen_relin();
  void keygen_rot(long step);
  const DevBuf& key(u64 g);

  HeCt encrypt_int(const i64* m_dev, int level, double scale, u64 nonce);
  HeCt encrypt(const double* z, int nz, int level, u64 nonce);
  std::vector<double> decrypt(const HeCt& c);

  HeCt add(const HeCt& a, const HeCt& b, bool sub);
  void add_into(HeCt& acc, const HeCt& b);
  HeCt drop(const HeCt& a, int level);
  HeCt rescale(const HeCt& a, int out_level = -1);
  DevBuf decompose(const u64* d, int level, int B = 1);
  HeCt hoisted(const HeCt& x, const u64* digits, u64 g);
  std::vector<HeCt> hoisted_multi(const HeCt& x, const u64* digits, const std::vector<u64>& gs);
  void hoisted_masked(const HeCt& x, const u64* digits, const std::vector<u64>& gs, const std::vector<u64*>& outs,
                      const std::vector<const u64*>& masks, bool accumulate);
  bool hoisted_masked_pair(const HeCt& x, const u64* dx, const std::vector<const u64*>& m1, const HeCt& y,
                           const u64* dy, const std::vector<const u64*>& m2, const std::vector<u64>& gs,
                           const std::vector<u64*>& outs);
  // consume: x's special-prime limbs (and q_l for moddown_rescale) may be
  // overwritten (x is a temporary the caller drops afterwards)
  // pack: the output's FP64 limbs may be stored packed (HeCt::packed says
  // whether they were: only on the fused, consuming path)
  HeCt moddown(const HeCt& x, int out_level = -1, bool consume = false, bool src_ready = false,
               const u64* rec = nullptr, bool pack = false);
  bool moddown_to(const HeCt& x, int out_level, u64* out, bool consume = false, bool src_ready = false,
                  const u64* rec = nullptr, bool pack = false);
  // ModDown and Rescale as one rounding by P q_l (a variant)
  HeCt moddown_rescale(const HeCt& x, int out_level = -1, bool consume = false, bool src_ready = false,
                       const u64* rec = nullptr, bool pack = false);
  // returns the digit records of the elements' ModDown sources when the
  // int8 lift takes them (element e's at rec + e * rec_stride), else empty
  DevBuf moddown_sources(const std::vector<HeCt*>& xs, bool with_rescale, size_t* rec_stride = nullptr);
  HeCt keyswitch(const u64* d, int level, u64 g_key, int B = 1);
  HeCt mult(const HeCt& a, const HeCt& b);
  HeCt rotate(const HeCt& x, long step);
  std::vector<HeCt> rotate_many(const HeCt& x, const std::vector<long>& steps);
  size_t rotate_workspace_bytes(int level, int B) const;
  void rotate_into(const HeCt& x, long step, u64* out, void* ws, size_t ws_bytes);
  HeCt pmult_int(const HeCt& a, const i64* m_dev, double pt_scale);
  void gather_limbs(u64* dst, const HeCt& x, int first, int count);
  HeCt stack(const std::vector<const HeCt*>& xs);
  std::vector<HeCt> unstack(const HeCt& x);

  // encoded plaintexts by key, cached; gen(i, v) gives the slot vector of
  // keys[i] (called only for keys not cached yet)
  using PtGen = std::function<void(size_t, std::vector<double>&)>;
  std::vector<const u64*> plaintexts(const std::vector<std::string>& keys, const PtGen& gen, int n2, int level,
                                     bool qp, double scale);
  HeCt lintrans(const HeCt& x, int kind, int n, int n1, double weight);
  // n1p: simple key substitution of the baby steps (section 4.2.1) when
  // 2 <= n1p < G.n1, else plain double hoisting
  HeCt lintrans_perm(const HeCt& x, const std::vector<int>& perm, const LtGeom& G, double weight,
                     const std::string& tag, int n1p = 0);
  HeCt lintrans_smpkeysub(const HeCt& x, int kind, int n, int n1, int n1p);
  HeCt apply_chain(const HeCt& x, const std::vector<DcdFactor>& fs, const std::string& tag);
  HeCt sigma_dcd(const HeCt& x, int n, int n1, int nprime);
  HeCt tau_dcd(const HeCt& x, int n, int n1, int nprime);
  HeCt matmul(const HeCt& a, const HeCt& b, int n, int n1z, int n1t, int npz, int npt, bool lazy = false,
              bool fused_rs = false, bool folded = false);
  // up to 8 products of one size, stacked, recorded once as a HIP graph (keyed
  // by the operands' buffers and the options) and replayed
  std::vector<HeCt> matmul_graph(const std::vector<const HeCt*>& a, const std::vector<const HeCt*>& b, int n,
                                 int n1z, int n1t, int npz, int npt, bool lazy, bool fused_rs, bool folded = false);
  void drop_graphs();
  // Products run together, one host thread each, taking turns on the
  // context: their key inner products are collected and launched as one
  // merged launch (launch_multsum_list) once every unfinished job has handed
  // one over.  Each job's residues are those it has alone.
  std::vector<HeCt> run_merged(const std::vector<std::function<HeCt()>>& jobs);
  void accumulate_tensors(DevBuf& acc3, bool& acc_set, const std::vector<HeCt>& Ak, const std::vector<HeCt>& Bk);
  HeCt relin_sum(const DevBuf& acc3, int level, double scale, int B);
  // pack: the A_k (with one rounding) and the ModDown'ed B_k may come out
  // packed, for the tensor sums alone
  std::vector<HeCt> matmul_side_a(const HeCt& ca, int n, int n1z, int npz, int out_level = -1,
                                  bool fused_rs = false, bool pack = false);
  std::vector<HeCt> matmul_side_b(const HeCt& cb, int n, int n1t, int npt, int out_level = -1, bool pack = false);
  // the A side with C^k's masks folded into Z: A_k = U_k a, one level
  std::vector<HeCt> matmul_side_a_folded(const HeCt& ca, int n, int n1z);
  void align_sides(std::vector<HeCt>& Ak, std::vector<HeCt>& Bk);
  void matmul_accumulate(HeCt& acc, bool& acc_set, const std::vector<HeCt>& Ak, const std::vector<HeCt>& Bk);
  std::vector<HeCt> covariance(const std::vector<const HeCt*>& x, int rb, int k, int n, u64 n_samples, int n1z,
                               int n1t, int n1g, int npz, int npt, bool lazy = false, bool fused_rs = false);
  // the same in parts: any split of the row blocks over cov_add calls gives
  // covariance's residues (the sums over row blocks are exact)
  CovState cov_begin(int k, int n, u64 n_samples, int n1z, int n1t, int n1g, int npz, int npt, bool lazy,
                     bool fused_rs);
  void cov_add(CovState& st, const std::vector<const HeCt*>& x, int rb);
  std::vector<HeCt> cov_end(CovState& st);
  // the same for a dataset that is not centred: X^T X / s - mu^T mu (section 5.2)
  std::vector<HeCt> covariance_uncentred(const std::vector<const HeCt*>& x, int rb, int k, int n, u64 n_samples,
                                         int n1z, int n1t, int n1g, int npz, int npt, bool lazy, bool fused_rs);

  // PowerMethod (section 6.1) and the interactive refresh
  DevBuf decrypt_int(const HeCt& c);
  HeCt refresh(const HeCt& c, u64 nonce);
  HeCt padd_int(const HeCt& a, const i64* m_dev);
  void power_step(std::vector<HeCt*>& cov, int k, int n, std::vector<HeCt*>& V, int axis, int tau, double x0,
                  bool last, bool goldschmidt, bool pack, const RefreshFn& refresh_fn, std::vector<HeCt>& v_out,
                  int& axis_out, HeCt& lambda_out, std::vector<HeCt>& vt_out);
  void eigen_shift(std::vector<HeCt*>& cov, int k, int n, HeCt& lambda, std::vector<HeCt*>& V,
                   std::vector<HeCt*>& VT, int axis, const RefreshFn& refresh_fn, std::vector<HeCt>& out);
};

struct he_ctx {
  mutable std::recursive_mutex mu;
  HeCtxImpl impl;
};
struct he_ct {
  he_ctx* ctx;
  HeCt ct;
};
struct he_cov {
  he_ctx* ctx;
  CovState st;
};
