// C ABI of the library (include/he_mi355x.h): argument checks, error
// translation and ownership; all computation is in runtime.hip / kernels.hip.
#include <cstdio>
#include <functional>
#include <map>
#include <mutex>
#include <set>

#include "runtime.h"

// Workspace of the allocation-free entry points: one copy per device, held
// until the process ends.  Host code never passes the array's name to a
// kernel (on the host it is a stand-in, not a device address): it uses the
// address hipGetSymbolAddress gives for the current device.
static __device__ __align__(256) u64 scratch[HE_NOALLOC_WS_BYTES / 8];

namespace {
template <class F>
he_status guard(F&& f) {
  try {
    f();
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) fail(HE_EDEVICE, std::string("HIP launch: ") + hipGetErrorString(e));
    return HE_OK;
  } catch (const HeError& e) {
    g_last_error = e.msg;
    return e.st;
  } catch (const std::bad_alloc&) {
    g_last_error = "host allocation failed";
    return HE_ENOMEM;
  } catch (const std::exception& e) {
    g_last_error = e.what();
    return HE_EINVAL;
  } catch (...) {
    g_last_error = "unknown error";
    return HE_EINVAL;
  }
}
// host-only calls: no HIP runtime query (they work without a device)
template <class F>
he_status guard_host(F&& f) {
  try {
    f();
    return HE_OK;
  } catch (const HeError& e) {
    g_last_error = e.msg;
    return e.st;
  } catch (const std::exception& e) {
    g_last_error = e.what();
    return HE_EINVAL;
  } catch (...) {
    g_last_error = "unknown error";
    return HE_EINVAL;
  }
}
void need(bool ok, const char* what) {
  if (!ok) fail(HE_EINVAL, what);
}
// one caller at a time per context (its stream, pool and caches are shared)
std::unique_lock<std::recursive_mutex> hold(const he_ctx* c) {
  need(c != nullptr, "null context");
  return std::unique_lock<std::recursive_mutex>(c->mu);
}
std::unique_lock<std::recursive_mutex> hold_ct(const he_ct* x) {
  need(x != nullptr, "null ciphertext");
  return hold(x->ctx);
}
he_ct* wrap(he_ctx* c, HeCt&& x) {
  he_ct* r = new he_ct;
  r->ctx = c;
  r->ct = std::move(x);
  return r;
}
void check_ct(const he_ctx* c, const he_ct* a) {
  need(a != nullptr, "null ciphertext");
  need(a->ctx == c, "ciphertext belongs to another context");
}
// device -> that device's address of `scratch`, looked up once per device
std::mutex g_ws_mu;
std::map<int, void*> g_ws_ptr;
void* workspace_of_current_device(int* dev_out) {
  int dev = 0;
  hip_check(hipGetDevice(&dev), "current device");
  *dev_out = dev;
  std::lock_guard<std::mutex> lk(g_ws_mu);
  auto it = g_ws_ptr.find(dev);
  if (it != g_ws_ptr.end()) return it->second;
  void* p = nullptr;
  hip_check(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)), "workspace address");
  if (!p) fail(HE_EDEVICE, "workspace address is null");
  g_ws_ptr[dev] = p;
  return p;
}
struct MmOpts {
  int n1z, n1t, npz, npt;
  bool lazy, fused, folded;
};
MmOpts opts_of(const he_matmul_opts* o, int d) {
  MmOpts m;
  m.n1z = (o && o->n1_z) ? (int)o->n1_z : default_n1(d);
  m.n1t = (o && o->n1_t) ? (int)o->n1_t : default_n1(d);
  m.npz = (o && o->nprime_z) ? (int)o->nprime_z : d - 1;
  m.npt = (o && o->nprime_t) ? (int)o->nprime_t : d - 1;
  if (m.npz > d - 1) m.npz = d - 1;
  if (m.npt > d - 1) m.npt = d - 1;
  m.lazy = o && (o->flags & HE_MM_LAZY_RELIN);
  m.fused = o && (o->flags & HE_MM_FUSED_RESCALE);
  m.folded = o && (o->flags & HE_MM_FOLDED);
  if (m.n1z < 1 || m.n1t < 1 || d % m.n1z || d % m.n1t) fail(HE_EINVAL, "baby-step counts must divide d");
  return m;
}
}  // namespace

extern "C" {

const char* he_last_error(void) { return g_last_error.c_str(); }

he_status he_ctx_create(const he_params* params, const he_device* dev, uint64_t seed, he_ctx** out) {
  return guard([&] {
    need(out != nullptr && params != nullptr, "null argument");
    *out = nullptr;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev == 0) {
      (void)hipGetLastError();
      fail(HE_EDEVICE, "no HIP device");
    }
    he_ctx* c = new he_ctx;
    try {
      c->impl.noalloc_ws = workspace_of_current_device(&c->impl.device);
      c->impl.init(params, dev, seed);
    } catch (...) {
      delete c;
      throw;
    }
    *out = c;
  });
}

he_status he_ctx_destroy(he_ctx* ctx) {
  return guard([&] { delete ctx; });
}

he_status he_ctx_moduli(const he_ctx* ctx, uint64_t* out, size_t cap, size_t* n) {
  return guard([&] {
    auto lk = hold(ctx);
    need(ctx != nullptr, "null context");
    const HeCtxImpl& c = ctx->impl;
    if (n) *n = (size_t)c.nmods;
    for (int k = 0; k < c.nmods && (size_t)k < cap; k++) out[k] = c.mods[k];
  });
}

he_status he_keygen(he_ctx* ctx, const int32_t* rot_steps, size_t n_steps) {
  return guard([&] {
    auto lk = hold(ctx);
    need(ctx != nullptr, "null context");
    HeCtxImpl& c = ctx->impl;
    c.drop_graphs();  // recorded products hold the keys' addresses
    c.keygen_secret();
    c.keygen_relin();
    for (size_t i = 0; i < n_steps; i++) c.keygen_rot(rot_steps[i]);
    hip_check(hipStreamSynchronize(c.stream), "keygen");
  });
}

he_status he_matmul_rot_steps(const he_ctx* ctx, uint32_t d, const he_matmul_opts* opts, int32_t* steps, size_t cap,
                              size_t* n) {
  return guard([&] {
    auto lk = hold(ctx);
    need(ctx != nullptr && d >= 2, "bad arguments");
    MmOpts m = opts_of(opts, (int)d);
    std::vector<long> s = matmul_steps((int)d, m.n1z, m.n1t, m.npz, m.npt, m.folded);
    if (n) *n = s.size();
    for (size_t i = 0; i < s.size() && i < cap; i++) steps[i] = (int32_t)s[i];
  });
}

he_status he_params_moduli(const he_params* p, uint64_t* moduli, uint64_t* psi, size_t cap) {
  return guard_host([&] {
    need(p && moduli && psi, "null argument");
    need(p->log_n >= 10 && p->log_n <= 16 && p->n_q >= 1 && p->n_q <= 48 && p->n_p >= 1 && p->n_p <= 4,
         "unsupported parameters");
    need(cap >= p->n_q + p->n_p, "buffers too small");
    std::vector<int> bits;
    for (u32 k = 0; k < p->n_q; k++) bits.push_back((int)p->q_bits[k]);
    for (u32 k = 0; k < p->n_p; k++) bits.push_back((int)p->p_bits[k]);
    for (int b : bits) need(b >= 30 && b <= 61, "prime sizes must be 30..61 bits");
    params_moduli((int)p->log_n, bits, moduli, psi);
  });
}

he_status he_lintrans_rot_steps(uint32_t kind, uint32_t d, uint32_t n1, uint32_t nprime, int32_t* steps, size_t cap,
                                size_t* n) {
  return guard_host([&] {
    need(kind <= 2 && d >= 2 && n1 >= 1 && d % n1 == 0, "bad arguments");
    std::set<long> s;
    lintrans_steps((int)kind, (int)d, (int)n1, nprime ? (int)nprime : (int)d - 1, s);
    if (n) *n = s.size();
    size_t i = 0;
    for (long v : s) {
      if (i < cap) steps[i] = (int32_t)v;
      i++;
    }
  });
}

he_status he_smpkeysub_rot_steps(uint32_t kind, uint32_t d, uint32_t n1, uint32_t n1p, int32_t* steps, size_t cap,
                                 size_t* n) {
  return guard_host([&] {
    need(kind <= 1 && d >= 2 && n1 >= 1 && d % n1 == 0 && n1p != 1, "bad arguments");
    std::set<long> s;
    bsgs_steps(make_perm((int)kind, (int)d), lt_geom((int)kind, (int)d, (int)n1), s, (int)n1p);
    if (n) *n = s.size();
    size_t i = 0;
    for (long v : s) {
      if (i < cap) steps[i] = (int32_t)v;
      i++;
    }
  });
}

he_status he_transpose_rot_steps(const he_ctx* ctx, uint32_t d, uint32_t n1, int32_t* steps, size_t cap, size_t* n) {
  return guard([&] {
    auto lk = hold(ctx);
    need(ctx != nullptr && d >= 2, "bad arguments");
    std::vector<long> s = transpose_steps((int)d, n1 ? (int)n1 : default_n1((int)d));
    if (n) *n = s.size();
    for (size_t i = 0; i < s.size() && i < cap; i++) steps[i] = (int32_t)s[i];
  });
}

he_status he_encode(he_ctx* ctx, const double* z, size_t n, double delta, int64_t* out) {
  return guard([&] {
    auto lk = hold(ctx);
    need(ctx && z && out && n > 0, "bad arguments");
    HeCtxImpl& c = ctx->impl;
    DevBuf m = c.encode_batch(z, (int)n, 1, delta);
    hip_check(hipMemcpyAsync(out, m.p, c.N * 8, hipMemcpyDeviceToHost, c.stream), "download");
    hip_check(hipStreamSynchronize(c.stream), "encode");
  });
}

he_status he_encrypt_slots(he_ctx* ctx, const double* z, size_t n, uint32_t level, uint64_t nonce, he_ct** out) {
  return guard([&] {
    auto lk = hold(ctx);
    need(ctx && z && out && n > 0, "bad arguments");
    *out = wrap(ctx, ctx->impl.encrypt(z, (int)n, (int)level, nonce));
  });
}

he_status he_encrypt_matrix(he_ctx* ctx, const double* a, uint32_t d, uint32_t level, uint64_t nonce, he_ct** out) {
  return guard([&] {
    auto lk = hold(ctx);
    need(ctx && a && out && d > 0, "bad arguments");
    need((u64)d * d <= ctx->impl.N / 2 && (ctx->impl.N / 2) % ((u64)d * d) == 0, "d*d must divide N/2");
    *out = wrap(ctx, ctx->impl.encrypt(a, (int)(d * d), (int)level, nonce));
  });
}

he_status he_decrypt(he_ctx* ctx, const he_ct* ct, double* out, size_t n) {
  return guard([&] {
    auto lk = hold(ctx);
    check_ct(ctx, ct);
    need(out != nullptr && n <= ctx->impl.N / 2, "bad output size");
    std::vector<double> z = ctx->impl.decrypt(ct->ct);
    std::copy(z.begin(), z.begin() + n, out);
  });
}

he_status he_ct_info(const he_ct* ct, uint32_t* level, double* scale) {
  return guard([&] {
    auto lk = hold_ct(ct);
    need(ct != nullptr, "null ciphertext");
    if (level) *level = (uint32_t)ct->ct.level;
    if (scale) *scale = ct->ct.scale;
  });
}

he_status he_ct_export(const he_ct* ct, uint64_t* host, size_t words, uint32_t* level, double* scale) {
  return guard([&] {
    auto lk = hold_ct(ct);
    need(ct != nullptr && host != nullptr, "null argument");
    need(words >= ct->ct.d.words, "host buffer too small");
    HeCtxImpl& c = ct->ctx->impl;
    hip_check(hipMemcpyAsync(host, ct->ct.d.p, ct->ct.d.words * 8, hipMemcpyDeviceToHost, c.stream), "export");
    hip_check(hipStreamSynchronize(c.stream), "export");
    if (level) *level = (uint32_t)ct->ct.level;
    if (scale) *scale = ct->ct.scale;
  });
}

he_status he_ct_import(he_ctx* ctx, const uint64_t* host, size_t words, uint32_t level, double scale, he_ct** out) {
  return guard([&] {
    auto lk = hold(ctx);
    need(ctx && host && out, "null argument");
    HeCtxImpl& c = ctx->impl;
    need((int)level <= c.L, "level out of range");
    HeCt x = c.ct_new((int)level, false, scale);
    need(words == x.d.words, "word count does not match 2*(level+1)*N");
    hip_check(hipMemcpyAsync(x.d.p, host, words * 8, hipMemcpyHostToDevice, c.stream), "import");
    hip_check(hipStreamSynchronize(c.stream), "import");
    *out = wrap(ctx, std::move(x));
  });
}

he_status he_ct_free(he_ct* ct) {
  return guard([&] {
    if (!ct) return;
    auto lk = hold(ct->ctx);
    delete ct;
  });
}

he_status he_add(he_ctx* ctx, const he_ct* a, const he_ct* b, he_ct** out) {
  return guard([&] {
    auto lk = hold(ctx);
    check_ct(ctx, a);
    check_ct(ctx, b);
    *out = wrap(ctx, ctx->impl.add(a->ct, b->ct, false));
  });
}
he_status he_sub(he_ctx* ctx, const he_ct* a, const he_ct* b, he_ct** out) {
  return guard([&] {
    auto lk = hold(ctx);
    check_ct(ctx, a);
    check_ct(ctx, b);
    *out = wrap(ctx, ctx->impl.add(a->ct, b->ct, true));
  });
}
he_status he_mult(he_ctx* ctx, const he_ct* a, const he_ct* b, he_ct** out) {
  return guard([&] {
    auto lk = hold(ctx);
    check_ct(ctx, a);
    check_ct(ctx, b);
    *out = wrap(ctx, ctx->impl.mult(a->ct, b->ct));
  });
}
he_status he_rescale(he_ctx* ctx, const he_ct* a, he_ct** out) {
  return guard([&] {
    auto lk = hold(ctx);
    check_ct(ctx, a);
    *out = wrap(ctx, ctx->impl.rescale(a->ct));
  });
}
he_status he_rotate(he_ctx* ctx, const he_ct* a, int32_t step, he_ct** out) {
  return guard([&] {
    auto lk = hold(ctx);
    check_ct(ctx, a);
    *out = wrap(ctx, ctx->impl.rotate(a->ct, step));
  });
}
he_status he_rotate_many(he_ctx* ctx, const he_ct* const* a, size_t count, const int32_t* steps, size_t nsteps,
                         he_ct** out) {
  return guard([&] {
    auto lk = hold(ctx);
    need(a && steps && out && count >= 1 && count <= 64 && nsteps >= 1 && nsteps <= 1024, "bad arguments");
    std::vector<const HeCt*> xs;
    for (size_t i = 0; i < count; i++) {
      check_ct(ctx, a[i]);
      xs.push_back(&a[i]->ct);
    }
    HeCtxImpl& c = ctx->impl;
    HeCt x = count == 1 ? c.ct_copy(*xs[0]) : c.stack(xs);
    std::vector<HeCt> rot = c.rotate_many(x, std::vector<long>(steps, steps + nsteps));
    std::vector<he_ct*> made;
    try {
      for (size_t r = 0; r < nsteps; r++) {
        std::vector<HeCt> parts = count == 1 ? std::vector<HeCt>{} : c.unstack(rot[r]);
        if (count == 1) parts.push_back(std::move(rot[r]));
        rot[r] = HeCt();
        for (size_t i = 0; i < count; i++) {
          made.push_back(wrap(ctx, std::move(parts[i])));
          out[i * nsteps + r] = made.back();
        }
      }
    } catch (...) {
      for (he_ct* m : made) delete m;
      throw;
    }
  });
}
he_status he_rotate_noalloc(he_ctx* ctx, const he_ct* a, int32_t step, he_ct* out) {
  return guard([&] {
    auto lk = hold(ctx);
    check_ct(ctx, a);
    check_ct(ctx, out);
    need(!a->ct.qp && !out->ct.qp, "rotation of an R_QP element");
    need(out->ct.level == a->ct.level && out->ct.B == a->ct.B,
         "the output must be a ciphertext at the input's level");
    HeCtxImpl& c = ctx->impl;
    const size_t need_bytes = c.rotate_workspace_bytes(a->ct.level, a->ct.B);
    if (need_bytes > HE_NOALLOC_WS_BYTES)
      fail(HE_EINVAL, "rotation at this level needs " + std::to_string(need_bytes) +
                          " bytes of workspace; the allocation-free entry point has " +
                          std::to_string((size_t)HE_NOALLOC_WS_BYTES));
    c.rotate_into(a->ct, step, out->ct.d.p, c.noalloc_ws, HE_NOALLOC_WS_BYTES);
    out->ct.scale = a->ct.scale;
  });
}
he_status he_rotate_workspace_bytes(const he_ctx* ctx, uint32_t level, size_t* bytes) {
  return guard_host([&] {
    need(ctx != nullptr && bytes != nullptr, "null argument");
    need((int)level <= ctx->impl.L, "level out of range");
    *bytes = ctx->impl.rotate_workspace_bytes((int)level, 1);
  });
}
he_status he_drop_level(he_ctx* ctx, const he_ct* a, uint32_t level, he_ct** out) {
  return guard([&] {
    auto lk = hold(ctx);
    check_ct(ctx, a);
    *out = wrap(ctx, ctx->impl.drop(a->ct, (int)level));
  });
}
he_status he_pmult_slots(he_ctx* ctx, const he_ct* a, const double* z, size_t n, double pt_scale, he_ct** out) {
  return guard([&] {
    auto lk = hold(ctx);
    check_ct(ctx, a);
    need(z && n > 0, "bad plaintext");
    HeCtxImpl& c = ctx->impl;
    DevBuf m = c.encode_batch(z, (int)n, 1, pt_scale);
    *out = wrap(ctx, c.pmult_int(a->ct, (const i64*)m.p, pt_scale));
  });
}

he_status he_lintrans(he_ctx* ctx, const he_ct* a, uint32_t kind, uint32_t d, uint32_t n1, double weight,
                      he_ct** out) {
  return guard([&] {
    auto lk = hold(ctx);
    check_ct(ctx, a);
    need(kind <= 2 && d >= 2, "bad transform");
    *out = wrap(ctx, ctx->impl.lintrans(a->ct, (int)kind, (int)d, n1 ? (int)n1 : default_n1((int)d), weight));
  });
}

he_status he_lintrans_dcd(he_ctx* ctx, const he_ct* a, uint32_t kind, uint32_t d, uint32_t n1, uint32_t nprime,
                          he_ct** out) {
  return guard([&] {
    auto lk = hold(ctx);
    check_ct(ctx, a);
    need(out != nullptr && kind <= 1 && d >= 2, "bad transform");
    const int n = (int)d, b1 = n1 ? (int)n1 : default_n1(n);
    need(n % b1 == 0, "baby-step count must divide d");
    const int np = (nprime == 0 || (int)nprime > n - 1) ? n - 1 : (int)nprime;
    HeCtxImpl& c = ctx->impl;
    *out = wrap(ctx, kind == 0 ? c.sigma_dcd(a->ct, n, b1, np) : c.tau_dcd(a->ct, n, b1, np));
  });
}

he_status he_lintrans_smpkeysub(he_ctx* ctx, const he_ct* a, uint32_t kind, uint32_t d, uint32_t n1, uint32_t n1p,
                                he_ct** out) {
  return guard([&] {
    auto lk = hold(ctx);
    check_ct(ctx, a);
    need(out != nullptr && kind <= 1 && d >= 2 && n1p != 1, "bad transform");
    const int n = (int)d, b1 = n1 ? (int)n1 : default_n1(n);
    need(n % b1 == 0, "baby-step count must divide d");
    *out = wrap(ctx, ctx->impl.lintrans_smpkeysub(a->ct, (int)kind, n, b1, (int)n1p));
  });
}

he_status he_matmul(he_ctx* ctx, const he_ct* a, const he_ct* b, uint32_t d, const he_matmul_opts* opts,
                    he_ct** out) {
  return guard([&] {
    auto lk = hold(ctx);
    check_ct(ctx, a);
    check_ct(ctx, b);
    need(out != nullptr && d >= 2, "bad arguments");
    HeCtxImpl& c = ctx->impl;
    MmOpts m = opts_of(opts, (int)d);
    hip_check(hipEventRecord(c.ev0, c.stream), "event");
    HeCt r = c.matmul(a->ct, b->ct, (int)d, m.n1z, m.n1t, m.npz, m.npt, m.lazy, m.fused, m.folded);
    hip_check(hipEventRecord(c.ev1, c.stream), "event");
    *out = wrap(ctx, std::move(r));
  });
}

he_status he_matmul_batch(he_ctx* ctx, const he_ct* const* a, const he_ct* const* b, const uint32_t* d,
                          size_t count, const he_matmul_opts* opts, he_ct** out) {
  return guard([&] {
    auto lk = hold(ctx);
    need(a && b && d && out, "null argument");
    HeCtxImpl& c = ctx->impl;
    for (size_t i = 0; i < count; i++) {
      check_ct(ctx, a[i]);
      check_ct(ctx, b[i]);
      out[i] = nullptr;
    }
    hip_check(hipEventRecord(c.ev0, c.stream), "event");
    if (opts && (opts->flags & HE_MM_GRAPH)) {
      need(opts->flags & HE_MM_BATCHED, "a recorded product must be batched");
      need(!(opts->flags & HE_MM_MERGED), "merged products are not recorded");
      need(count >= 1 && count <= 8, "a recorded product takes 1 to 8 pairs");
      need(!prof_enabled(), "no recording while the kernel profile is enabled");
      std::vector<const HeCt*> xa, xb;
      for (size_t k = 0; k < count; k++) {
        need(d[k] == d[0], "a recorded product takes one matrix size");
        xa.push_back(&a[k]->ct);
        xb.push_back(&b[k]->ct);
      }
      MmOpts m = opts_of(opts, (int)d[0]);
      std::vector<HeCt> parts = c.matmul_graph(xa, xb, (int)d[0], m.n1z, m.n1t, m.npz, m.npt, m.lazy, m.fused, m.folded);
      for (size_t k = 0; k < count; k++) out[k] = wrap(ctx, std::move(parts[k]));
      hip_check(hipEventRecord(c.ev1, c.stream), "event");
      return;
    }
    try {
      if (opts && (opts->flags & HE_MM_MERGED)) {
        // products of equal d, level and scales stacked (up to 8, wherever
        // they stand in the list); the stacks run together with their key
        // inner products merged into shared launches
        std::vector<std::vector<size_t>> stacks;
        for (size_t i = 0; i < count; i++) {
          bool placed = false;
          for (auto& st : stacks) {
            const size_t j = st[0];
            if (st.size() < 8 && d[j] == d[i] && a[j]->ct.level == a[i]->ct.level &&
                b[j]->ct.level == b[i]->ct.level && a[j]->ct.scale == a[i]->ct.scale &&
                b[j]->ct.scale == b[i]->ct.scale) {
              st.push_back(i);
              placed = true;
              break;
            }
          }
          if (!placed) stacks.push_back({i});
        }
        std::vector<std::function<HeCt()>> jobs;
        for (const auto& st : stacks) {
          jobs.push_back([&, st]() {
            std::vector<const HeCt*> xa, xb;
            for (size_t k : st) {
              xa.push_back(&a[k]->ct);
              xb.push_back(&b[k]->ct);
            }
            MmOpts m = opts_of(opts, (int)d[st[0]]);
            HeCt sa = st.size() == 1 ? c.ct_copy(*xa[0]) : c.stack(xa);
            HeCt sb = st.size() == 1 ? c.ct_copy(*xb[0]) : c.stack(xb);
            return c.matmul(sa, sb, (int)d[st[0]], m.n1z, m.n1t, m.npz, m.npt, m.lazy, m.fused, m.folded);
          });
        }
        std::vector<HeCt> res = c.run_merged(jobs);
        for (size_t s_ = 0; s_ < stacks.size(); s_++) {
          std::vector<HeCt> parts = stacks[s_].size() == 1 ? std::vector<HeCt>{} : c.unstack(res[s_]);
          if (stacks[s_].size() == 1) parts.push_back(std::move(res[s_]));
          for (size_t k = 0; k < stacks[s_].size(); k++) out[stacks[s_][k]] = wrap(ctx, std::move(parts[k]));
        }
      } else if (opts && (opts->flags & HE_MM_BATCHED)) {
        // runs of equal d stacked into batches of up to 8: every launch of the
        // plan then serves the whole batch (keys read once per batch)
        size_t i = 0;
        while (i < count) {
          size_t j = i + 1;
          while (j < count && j - i < 8 && d[j] == d[i] && a[j]->ct.level == a[i]->ct.level &&
                 a[j]->ct.scale == a[i]->ct.scale && b[j]->ct.scale == b[i]->ct.scale)
            j++;
          std::vector<const HeCt*> xa, xb;
          for (size_t k = i; k < j; k++) {
            xa.push_back(&a[k]->ct);
            xb.push_back(&b[k]->ct);
          }
          MmOpts m = opts_of(opts, (int)d[i]);
          HeCt sa = c.stack(xa), sb = c.stack(xb);
          HeCt r = c.matmul(sa, sb, (int)d[i], m.n1z, m.n1t, m.npz, m.npt, m.lazy, m.fused, m.folded);
          std::vector<HeCt> parts = c.unstack(r);
          for (size_t k = i; k < j; k++) out[k] = wrap(ctx, std::move(parts[k - i]));
          i = j;
        }
      } else {
        for (size_t i = 0; i < count; i++) {
          MmOpts m = opts_of(opts, (int)d[i]);
          out[i] = wrap(ctx, c.matmul(a[i]->ct, b[i]->ct, (int)d[i], m.n1z, m.n1t, m.npz, m.npt, m.lazy, m.fused, m.folded));
        }
      }
    } catch (...) {
      for (size_t i = 0; i < count; i++) {
        delete out[i];
        out[i] = nullptr;
      }
      throw;
    }
    hip_check(hipEventRecord(c.ev1, c.stream), "event");
  });
}

he_status he_covariance(he_ctx* ctx, const he_ct* const* x, uint32_t row_blocks, uint32_t k, uint32_t d,
                        uint64_t n_samples, const he_matmul_opts* opts, he_ct** cov) {
  return guard([&] {
    auto lk = hold(ctx);
    need(x && cov && row_blocks > 0 && k > 0 && d >= 2 && n_samples > 0, "bad arguments");
    std::vector<const HeCt*> xs;
    for (uint32_t i = 0; i < row_blocks * k; i++) {
      check_ct(ctx, x[i]);
      xs.push_back(&x[i]->ct);
    }
    MmOpts m = opts_of(opts, (int)d);
    need(!m.folded, "the covariance takes the three-level product");
    HeCtxImpl& c = ctx->impl;
    hip_check(hipEventRecord(c.ev0, c.stream), "event");
    std::vector<HeCt> r =
        (opts && (opts->flags & HE_COV_UNCENTRED))
            ? c.covariance_uncentred(xs, (int)row_blocks, (int)k, (int)d, n_samples, m.n1z, m.n1t, default_n1((int)d),
                                     m.npz, m.npt, m.lazy, m.fused)
            : c.covariance(xs, (int)row_blocks, (int)k, (int)d, n_samples, m.n1z, m.n1t, default_n1((int)d), m.npz,
                           m.npt, m.lazy, m.fused);
    hip_check(hipEventRecord(c.ev1, c.stream), "event");
    for (uint32_t i = 0; i < k * k; i++) cov[i] = wrap(ctx, std::move(r[i]));
  });
}

he_status he_covariance_begin(he_ctx* ctx, uint32_t k, uint32_t d, uint64_t n_samples, const he_matmul_opts* opts,
                              he_cov** st) {
  return guard([&] {
    auto lk = hold(ctx);
    need(st && k > 0 && d >= 2 && n_samples > 0, "bad arguments");
    need(!(opts && (opts->flags & HE_COV_UNCENTRED)), "the covariance in parts takes a centred dataset");
    MmOpts m = opts_of(opts, (int)d);
    need(!m.folded, "the covariance takes the three-level product");
    he_cov* c = new he_cov;
    c->ctx = ctx;
    c->st = ctx->impl.cov_begin((int)k, (int)d, n_samples, m.n1z, m.n1t, default_n1((int)d), m.npz, m.npt, m.lazy,
                                m.fused);
    *st = c;
  });
}

he_status he_covariance_add(he_cov* st, const he_ct* const* x, uint32_t row_blocks) {
  return guard([&] {
    need(st != nullptr, "null covariance state");
    he_ctx* ctx = st->ctx;
    auto lk = hold(ctx);
    need(x && row_blocks > 0, "bad arguments");
    std::vector<const HeCt*> xs;
    for (uint32_t i = 0; i < row_blocks * (uint32_t)st->st.k; i++) {
      check_ct(ctx, x[i]);
      xs.push_back(&x[i]->ct);
    }
    HeCtxImpl& c = ctx->impl;
    hip_check(hipEventRecord(c.ev0, c.stream), "event");
    c.cov_add(st->st, xs, (int)row_blocks);
    hip_check(hipEventRecord(c.ev1, c.stream), "event");
  });
}

he_status he_covariance_end(he_cov* st, he_ct** cov) {
  return guard([&] {
    need(st != nullptr && cov != nullptr, "bad arguments");
    he_ctx* ctx = st->ctx;
    auto lk = hold(ctx);
    HeCtxImpl& c = ctx->impl;
    hip_check(hipEventRecord(c.ev0, c.stream), "event");
    std::vector<HeCt> r = c.cov_end(st->st);
    hip_check(hipEventRecord(c.ev1, c.stream), "event");
    for (size_t i = 0; i < r.size(); i++) cov[i] = wrap(ctx, std::move(r[i]));
  });
}

he_status he_covariance_free(he_cov* st) {
  return guard([&] {
    if (!st) return;
    auto lk = hold(st->ctx);
    delete st;
  });
}

// ---------------------------------------------------------------------------
// PowerMethod (section 6.1) and the interactive refresh
// ---------------------------------------------------------------------------
he_status he_refresh(he_ctx* ctx, he_ct* ct, uint64_t nonce) {
  return guard([&] {
    auto lk = hold(ctx);
    check_ct(ctx, ct);
    ct->ct = ctx->impl.refresh(ct->ct, nonce);
  });
}

he_status he_power_rot_steps(uint32_t d, int32_t* steps, size_t cap, size_t* n) {
  return guard_host([&] {
    need(d >= 2 && (d & (d - 1)) == 0 && n != nullptr, "d must be a power of two");
    std::set<long> s;
    for (long i = 1; i < (long)d; i <<= 1) {
      s.insert(i);
      s.insert(-i);
      s.insert(i * (long)d);
    }
    *n = s.size();
    size_t i = 0;
    for (long v : s) {
      if (i < cap) steps[i] = (int32_t)v;
      i++;
    }
  });
}

namespace {
RefreshFn make_refresh(he_ctx* ctx, he_refresh_fn fn, void* user) {
  return [ctx, fn, user](HeCt& x) {
    if (!fn) fail(HE_ENEEDREFRESH, "a ciphertext ran out of levels and no refresh callback was given");
    he_ct tmp;
    tmp.ctx = ctx;
    tmp.ct = std::move(x);
    he_status st = fn(&tmp, user);
    x = std::move(tmp.ct);
    if (st != HE_OK) fail(st, "refresh callback failed");
    if (x.level < 1) fail(HE_ENEEDREFRESH, "refresh callback left the ciphertext without levels");
  };
}
}  // namespace

he_status he_power_step(he_ctx* ctx, he_ct* const* cov, uint32_t k, uint32_t d, he_ct* const* v, uint32_t axis,
                        uint32_t newton_iters, double taylor_x0, uint32_t taylor_order, int last, uint32_t flags,
                        he_refresh_fn refresh, void* user, he_ct** v_out, uint32_t* axis_out, he_ct** lambda_out,
                        he_ct** vt_out) {
  return guard([&] {
    auto lk = hold(ctx);
    need(cov && v && axis_out && k > 0, "null argument");
    need((flags & ~(HE_PM_GOLDSCHMIDT | HE_PM_PACK_REFRESH)) == 0, "unknown power-step flag");
    need(taylor_order == 1, "only the order-1 TaylorInit is implemented");
    need(taylor_x0 > 0, "Taylor point must be positive");
    need(last ? (lambda_out && vt_out) : (v_out != nullptr), "null output");
    std::vector<HeCt*> C, V;
    for (uint32_t i = 0; i < k * k; i++) {
      check_ct(ctx, cov[i]);
      C.push_back(&cov[i]->ct);
    }
    for (uint32_t i = 0; i < k; i++) {
      check_ct(ctx, v[i]);
      V.push_back(&v[i]->ct);
    }
    std::vector<HeCt> vo, vto;
    HeCt lam;
    int ax = 0;
    ctx->impl.power_step(C, (int)k, (int)d, V, (int)axis, (int)newton_iters, taylor_x0, last != 0,
                         (flags & HE_PM_GOLDSCHMIDT) != 0, (flags & HE_PM_PACK_REFRESH) != 0,
                         make_refresh(ctx, refresh, user), vo, ax, lam, vto);
    *axis_out = (uint32_t)ax;
    if (last) {
      *lambda_out = wrap(ctx, std::move(lam));
      for (uint32_t i = 0; i < k; i++) vt_out[i] = wrap(ctx, std::move(vto[i]));
    } else {
      for (uint32_t i = 0; i < k; i++) v_out[i] = wrap(ctx, std::move(vo[i]));
    }
  });
}

he_status he_eigen_shift(he_ctx* ctx, he_ct* const* cov, uint32_t k, uint32_t d, he_ct* lambda, he_ct* const* v,
                         he_ct* const* vt, uint32_t axis, he_refresh_fn refresh, void* user, he_ct** cov_out) {
  return guard([&] {
    auto lk = hold(ctx);
    need(cov && v && vt && lambda && cov_out && k > 0 && axis <= 1, "bad arguments");
    check_ct(ctx, lambda);
    std::vector<HeCt*> C, V, VT;
    for (uint32_t i = 0; i < k * k; i++) {
      check_ct(ctx, cov[i]);
      C.push_back(&cov[i]->ct);
    }
    for (uint32_t i = 0; i < k; i++) {
      check_ct(ctx, v[i]);
      check_ct(ctx, vt[i]);
      V.push_back(&v[i]->ct);
      VT.push_back(&vt[i]->ct);
    }
    std::vector<HeCt> out;
    ctx->impl.eigen_shift(C, (int)k, (int)d, lambda->ct, V, VT, (int)axis, make_refresh(ctx, refresh, user), out);
    for (uint32_t i = 0; i < k * k; i++) cov_out[i] = wrap(ctx, std::move(out[i]));
  });
}

he_status he_knob_set(const char* name, int32_t value) {
  return guard_host([&] {
    need(name != nullptr, "null name");
    if (!knob_set(name, value)) fail(HE_EINVAL, std::string("unknown knob or value out of range: ") + name);
  });
}
he_status he_knob_get(const char* name, int32_t* value) {
  return guard_host([&] {
    need(name != nullptr && value != nullptr, "null argument");
    int v = 0;
    if (!knob_get(name, &v)) fail(HE_EINVAL, std::string("unknown knob: ") + name);
    *value = v;
  });
}

he_status he_sync(he_ctx* ctx) {
  return guard([&] {
    auto lk = hold(ctx);
    need(ctx != nullptr, "null context");
    hip_check(hipStreamSynchronize(ctx->impl.stream), "sync");
  });
}

he_status he_mem_info(const he_ctx* ctx, size_t* live, size_t* cached, size_t* peak) {
  return guard([&] {
    auto lk = hold(ctx);
    need(ctx != nullptr, "null context");
    if (live) *live = ctx->impl.pool.bytes_live;
    if (cached) *cached = ctx->impl.pool.bytes_cached;
    if (peak) *peak = ctx->impl.pool.peak;
  });
}

he_status he_modmul_peak(uint32_t kind, uint64_t iters, uint32_t blocks, double* products_per_s, double* ms) {
  return guard([&] {
    need(products_per_s != nullptr, "null argument");
    modmul_peak((int)kind, iters, (int)blocks, products_per_s, ms);
  });
}

he_status he_device_memory(size_t* free_bytes, size_t* total_bytes) {
  return guard([&] {
    need(free_bytes && total_bytes, "null argument");
    hip_check(hipMemGetInfo(free_bytes, total_bytes), "memory info");
  });
}

he_status he_trim(he_ctx* ctx) {
  return guard([&] {
    auto lk = hold(ctx);
    need(ctx != nullptr, "null context");
    hip_check(hipStreamSynchronize(ctx->impl.stream), "sync");
    ctx->impl.drop_graphs();
    ctx->impl.pool.trim();
    ctx->impl.pool.peak = ctx->impl.pool.bytes_live;
  });
}

he_status he_ntt_limbs(he_ctx* ctx, const uint64_t* in, uint64_t* out, size_t nlimbs, const int32_t* mod_idx,
                       int inverse) {
  return guard([&] {
    auto lk = hold(ctx);
    need(ctx && in && out && mod_idx && nlimbs > 0 && nlimbs <= 960, "bad arguments");
    HeCtxImpl& c = ctx->impl;
    LimbMap m;
    m.n = (int)nlimbs;
    for (size_t k = 0; k < nlimbs; k++) {
      need(mod_idx[k] >= 0 && mod_idx[k] < c.nmods, "modulus index out of range");
      m.idx[k] = (short)mod_idx[k];
    }
    for (size_t k = 0; k < nlimbs; k++)
      for (u64 i = 0; i < c.N; i++) need(in[k * c.N + i] < c.mods[mod_idx[k]], "residue not reduced");
    DevBuf d(&c.pool, nlimbs * c.N);
    hip_check(hipMemcpyAsync(d.p, in, nlimbs * c.N * 8, hipMemcpyHostToDevice, c.stream), "upload");
    launch_ntt(c.T, d.p, (int)nlimbs, m, inverse != 0, c.stream);
    hip_check(hipMemcpyAsync(out, d.p, nlimbs * c.N * 8, hipMemcpyDeviceToHost, c.stream), "download");
    hip_check(hipStreamSynchronize(c.stream), "ntt");
  });
}

he_status he_automorph_limbs(he_ctx* ctx, const uint64_t* in, uint64_t* out, size_t nlimbs, uint64_t galois) {
  return guard([&] {
    auto lk = hold(ctx);
    need(ctx && in && out && nlimbs > 0, "bad arguments");
    HeCtxImpl& c = ctx->impl;
    need(galois % 2 == 1 && galois < 2 * c.N, "Galois element must be odd and below 2N");
    DevBuf a(&c.pool, nlimbs * c.N), b(&c.pool, nlimbs * c.N);
    hip_check(hipMemcpyAsync(a.p, in, nlimbs * c.N * 8, hipMemcpyHostToDevice, c.stream), "upload");
    launch_automorph(c.T, b.p, a.p, (int)nlimbs, galois, c.stream);
    hip_check(hipMemcpyAsync(out, b.p, nlimbs * c.N * 8, hipMemcpyDeviceToHost, c.stream), "download");
    hip_check(hipStreamSynchronize(c.stream), "automorph");
  });
}

he_status he_hoisted_rotate_export(he_ctx* ctx, const he_ct* a, int32_t step, uint64_t* host, size_t words) {
  return guard([&] {
    auto lk = hold(ctx);
    check_ct(ctx, a);
    HeCtxImpl& c = ctx->impl;
    u64 g = c.galois(step);
    DevBuf dig;
    if (g != 1) dig = c.decompose(a->ct.poly(1), a->ct.level);
    HeCt h = c.hoisted(a->ct, dig.p, g);
    need(words >= h.d.words, "host buffer too small");
    hip_check(hipMemcpyAsync(host, h.d.p, h.d.words * 8, hipMemcpyDeviceToHost, c.stream), "download");
    hip_check(hipStreamSynchronize(c.stream), "hoisted");
  });
}

he_status he_last_op_ms(const he_ctx* ctx, double* ms) {
  return guard([&] {
    auto lk = hold(ctx);
    need(ctx && ms, "null argument");
    float f = 0;
    hip_check(hipEventSynchronize(ctx->impl.ev1), "event");
    hip_check(hipEventElapsedTime(&f, ctx->impl.ev0, ctx->impl.ev1), "event");
    *ms = f;
  });
}

he_status he_profile_enable(he_ctx* ctx, int on) {
  return guard([&] {
    auto lk = hold(ctx);
    need(ctx != nullptr, "null context");
    hip_check(hipStreamSynchronize(ctx->impl.stream), "sync");
    prof_enable(on != 0);
  });
}

he_status he_profile_read(he_ctx* ctx, const char* family, double* total_ms, uint64_t* launches, double* bytes) {
  return guard([&] {
    auto lk = hold(ctx);
    need(ctx && family && total_ms && launches, "null argument");
    hip_check(hipStreamSynchronize(ctx->impl.stream), "sync");
    u64 n = 0;
    double b = 0;
    prof_read(family, total_ms, &n, &b);
    *launches = n;
    if (bytes) *bytes = b;
  });
}

he_status he_profile_read_ops(he_ctx* ctx, const char* family, double* modmuls_f64, double* modmuls_int,
                              double* unit_bytes) {
  return guard([&] {
    auto lk = hold(ctx);
    need(ctx && family && modmuls_f64 && modmuls_int, "null argument");
    double u = 0;
    prof_read_ops(family, modmuls_f64, modmuls_int, &u);
    if (unit_bytes) *unit_bytes = u;
  });
}

he_status he_op_counts(const he_ctx* ctx, uint64_t* decompose, uint64_t* multsum, uint64_t* moddown) {
  return guard([&] {
    auto lk = hold(ctx);
    need(ctx != nullptr, "null context");
    if (decompose) *decompose = (uint64_t)ctx->impl.n_decompose;
    if (multsum) *multsum = (uint64_t)ctx->impl.n_multsum;
    if (moddown) *moddown = (uint64_t)ctx->impl.n_moddown;
  });
}

}  // extern "C"
