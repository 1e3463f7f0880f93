// C ABI (include/secpe.h) over the runtime.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/secpe.h"
#include "boot_tables.h"
#include "runtime.h"

struct secpe_ctx {
  secpe::Ctx c;
  bool own_stream = false;
  const double* evk = nullptr;
  std::vector<const double*> key_list;
};

// The key owner's side of the refresh stand-in: a reference to the secret key
// (caller-owned device memory) and the parameters it belongs to.  Contexts
// never store it; every evaluation that may refresh is handed one.
struct secpe_key_owner {
  const double* sk = nullptr;
  int device = 0;
  std::vector<uint64_t> mod;
};

using namespace secpe;

static thread_local std::string g_err;

static int set_err(int code, const std::string& msg) {
  g_err = msg;
  return code;
}

extern "C" const char* secpe_last_error(void) { return g_err.c_str(); }

extern "C" const char* secpe_strerror(int code) {
  switch (code) {
    case SECPE_OK: return "success";
    case SECPE_EINVAL: return "invalid argument or parameter set";
    case SECPE_ENOMEM: return "workspace or device memory too small";
    case SECPE_ENOLEVEL: return "modulus chain exhausted: a key owner or bootstrapping is needed";
    case SECPE_ENOKEY: return "no switching key for a needed rotation";
    case SECPE_EDEVICE: return "HIP device error";
    default: return "unknown error code";
  }
}

#define CHECK_CTX(ctx) \
  if (!(ctx)) return set_err(SECPE_EINVAL, "null context")

static int hip_fail(const char* where, hipError_t e) {
  return set_err(SECPE_EDEVICE, std::string(where) + ": " + hipGetErrorString(e));
}

static int ensure_buffer(Ctx& c, char** buf, size_t* cap, size_t need) {
  if (*cap >= need && *buf) return 0;
  if (c.stream) (void)hipStreamSynchronize(c.stream);
  if (*buf) (void)hipFree(*buf);
  *buf = nullptr;
  *cap = 0;
  size_t n = std::max(need, (size_t)1 << 20);
  hipError_t e = hipMalloc((void**)buf, n);
  if (e != hipSuccess) {
    *buf = nullptr;
    return hip_fail("hipMalloc", e);
  }
  *cap = n;
  return 0;
}

// ---------------------------------------------------------------------------
// Scratch of the evaluation that allocates nothing (secpe_eval_argmax_noalloc):
// one device-global array per GPU holds that call's workspace and descriptor
// arena.  In host code the array's name is no device address: each device's
// copy is looked up once, with that device current, at context creation
// (hipGetSymbolAddress) and only the looked-up pointer is used afterwards.
// ---------------------------------------------------------------------------
static __device__ __align__(256) char scratch[SECPE_NOALLOC_SCRATCH_BYTES];
static std::mutex g_scratch_mu;
static std::map<int, char*> g_scratch_ptr;   // device -> address of its copy of 'scratch'

// Record the current device's scratch address (idempotent); 'device' is current.
static int scratch_lookup(int device) {
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_ptr.count(device)) return 0;
  void* p = nullptr;
  hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !p) return hip_fail("hipGetSymbolAddress(scratch)", e);
  g_scratch_ptr[device] = (char*)p;
  return 0;
}

static char* scratch_ptr(int device) {
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  auto it = g_scratch_ptr.find(device);
  return it == g_scratch_ptr.end() ? nullptr : it->second;
}

// The secret an evaluation may refresh with: null without a key owner; an
// error when the owner belongs to other parameters or another device.
static int owner_sk(const secpe_ctx* x, const secpe_key_owner* o, const double** sk) {
  *sk = nullptr;
  if (!o) return 0;
  if (!o->sk || o->device != x->c.device || o->mod != x->c.mod)
    return set_err(SECPE_EINVAL, "key owner has other parameters or another device");
  *sk = o->sk;
  return 0;
}

// Build with 'fn' into the context arena (growing it when needed) and submit.
template <class F>
static int run_build(secpe_ctx* x, char* ws, size_t ws_bytes, F fn, bool record = true) {
  Ctx& c = x->c;
  for (int attempt = 0; attempt < 3; ++attempt) {
    Builder b(c, ws, ws_bytes, c.arena, c.arena_bytes, false);
    fn(b);
    if (b.err_code) return set_err(b.err_code, b.err);
    if (b.arena_overflow() || !c.arena) {
      int rc = ensure_buffer(c, &c.arena, &c.arena_bytes, b.blob_bytes() + b.blob_bytes() / 4 + 4096);
      if (rc) return rc;
      continue;
    }
    int rc = submit(c, b, c.arena, c.arena_bytes);
    if (rc) return set_err(SECPE_EDEVICE, "kernel submission failed");
    if (record) {
      memcpy(c.counters, b.counters, sizeof(c.counters));
      c.ks_alg_limbs = b.ks_alg_limbs;
    }
    return 0;
  }
  return set_err(SECPE_ENOMEM, "descriptor arena did not converge");
}

// client scratch sized by a dry run
template <class F>
static int run_client(secpe_ctx* x, F fn) {
  Ctx& c = x->c;
  Builder dry(c, (char*)(uintptr_t)0x100000000000ull, (size_t)1 << 44, (char*)(uintptr_t)0x400000000000ull, (size_t)1 << 40, true);
  fn(dry);
  if (dry.err_code) return set_err(dry.err_code, dry.err);
  int rc = ensure_buffer(c, &c.client, &c.client_bytes, dry.need_bytes() + 4096);
  if (rc) return rc;
  return run_build(x, c.client, c.client_bytes, fn, false);
}

static int sync(Ctx& c) {
  hipError_t e = c.stream ? hipStreamSynchronize(c.stream) : hipDeviceSynchronize();
  if (e != hipSuccess) return hip_fail("synchronize", e);
  return 0;
}

// ---------------------------------------------------------------------------
extern "C" int secpe_ctx_create(const secpe_params* p, int device, void* stream, secpe_ctx** out) {
  if (!p || !out) return set_err(SECPE_EINVAL, "null argument");
  *out = nullptr;
  if (p->log_n < 10 || p->log_n > 16) return set_err(SECPE_EINVAL, "log_n must be in [10, 16]");
  if (p->n_q < 2 || p->n_p < 1 || p->n_p > 16) return set_err(SECPE_EINVAL, "need n_q >= 2 and 1 <= n_p <= 16");
  if (p->q_bits < 20 || p->q_bits > 50 || p->p_bits < 20 || p->p_bits > 51)
    return set_err(SECPE_EINVAL, "prime sizes must keep every modulus below 2^51");
  if (p->dg < 0 || p->df < 0 || p->dg + p->df < 1 || p->min_level < 1 || p->log_scale < 10 || p->log_scale > 60)
    return set_err(SECPE_EINVAL, "bad Sign or scale parameters");
  if (p->refresh_level < 0) return set_err(SECPE_EINVAL, "refresh_level must be >= 0");
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev)
    return set_err(SECPE_EDEVICE, "no such HIP device");
  secpe_ctx* x = new secpe_ctx();
  if (hipSetDevice(device) != hipSuccess) { delete x; return set_err(SECPE_EDEVICE, "hipSetDevice failed"); }
  hipStream_t s = (hipStream_t)stream;
  if (!s) {
    if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) {
      delete x;
      return set_err(SECPE_EDEVICE, "stream creation failed");
    }
    x->own_stream = true;
  }
  int rc = build_context(x->c, p->log_n, p->n_q, p->q_bits, p->n_p, p->p_bits, p->log_scale, p->dg, p->df,
                         p->min_level, p->refresh_level, device, s);
  if (rc) {
    destroy_context(x->c);
    if (x->own_stream) (void)hipStreamDestroy(s);
    delete x;
    return set_err(SECPE_EDEVICE, "context tables could not be built");
  }
  if ((x->c.mod.back() >> 51) != 0) {
    secpe_ctx_destroy(x);
    return set_err(SECPE_EINVAL, "a modulus reached 2^51");
  }
  // set-up for secpe_eval_argmax_noalloc: this device's scratch address and a
  // pinned staging buffer its descriptor blobs fit in
  rc = scratch_lookup(device);
  if (!rc) {
    x->c.staging_bytes = SECPE_NOALLOC_BLOB_BYTES;
    if (hipHostMalloc((void**)&x->c.staging, x->c.staging_bytes, hipHostMallocDefault) != hipSuccess) {
      x->c.staging = nullptr;
      x->c.staging_bytes = 0;
      rc = set_err(SECPE_EDEVICE, "pinned staging allocation failed");
    }
  }
  if (rc) {
    secpe_ctx_destroy(x);
    return rc;
  }
  *out = x;
  return 0;
}

extern "C" void secpe_ctx_destroy(secpe_ctx* x) {
  if (!x) return;
  hipStream_t s = x->c.stream;
  destroy_context(x->c);
  if (x->own_stream && s) (void)hipStreamDestroy(s);
  delete x;
}

extern "C" int secpe_primes(const secpe_ctx* x, uint64_t* out, int cap) {
  CHECK_CTX(x);
  const int n = (int)x->c.mod.size();
  for (int i = 0; i < n && i < cap; ++i) out[i] = x->c.mod[i];
  return n;
}
extern "C" int secpe_slots(const secpe_ctx* x) { return x ? x->c.N / 2 : 0; }
extern "C" size_t secpe_ct_bytes(const secpe_ctx* x) { return x ? x->c.ct_bytes() : 0; }
extern "C" size_t secpe_sk_bytes(const secpe_ctx* x) { return x ? x->c.sk_bytes() : 0; }
extern "C" size_t secpe_key_bytes(const secpe_ctx* x) { return x ? x->c.key_bytes() : 0; }
extern "C" uint64_t secpe_galois_elt(const secpe_ctx* x, int64_t step) { return x ? x->c.galois(step) : 0; }

extern "C" int secpe_argmax_steps(const secpe_ctx* x, int k_max, int c_max, int64_t* out, int cap) {
  CHECK_CTX(x);
  const int slots = x->c.N / 2;
  const int cpm = 1 << ilog2_ceil(std::max(1, c_max));
  const int kpm = 1 << ilog2_ceil(std::max(1, k_max));
  std::vector<int64_t> st;
  for (int cp = 1; cp <= cpm; cp <<= 1) {
    st.push_back(slots - cp);
    for (int i = 1; i < kpm; i <<= 1) st.push_back((int64_t)cp * i);
  }
  for (int j = 1; j < cpm; j <<= 1) st.push_back(j);
  std::sort(st.begin(), st.end());
  st.erase(std::unique(st.begin(), st.end()), st.end());
  st.erase(std::remove_if(st.begin(), st.end(), [&](int64_t v) { return v % slots == 0; }), st.end());
  for (size_t i = 0; i < st.size() && (int)i < cap; ++i) out[i] = st[i];
  return (int)st.size();
}

extern "C" int secpe_phoenix_steps(const secpe_ctx* x, int k_max, int c, int64_t* out, int cap) {
  CHECK_CTX(x);
  if (c < 2) return set_err(SECPE_EINVAL, "need C >= 2");
  const int slots = x->c.N / 2;
  std::vector<int64_t> st(256);
  int n = secpe_argmax_steps(x, k_max, c, st.data(), (int)st.size());
  if (n < 0) return n;
  st.resize(n);
  for (int i = 1; i < c; ++i) st.push_back(i);
  st.push_back(slots - c);
  std::sort(st.begin(), st.end());
  st.erase(std::unique(st.begin(), st.end()), st.end());
  st.erase(std::remove_if(st.begin(), st.end(), [&](int64_t v) { return v % slots == 0; }), st.end());
  for (size_t i = 0; i < st.size() && (int)i < cap; ++i) out[i] = st[i];
  return (int)st.size();
}

// ---------------------------------------------------------------------------
// keys
// ---------------------------------------------------------------------------
extern "C" int secpe_keygen(secpe_ctx* x, uint64_t seed, const int64_t* steps, int n_steps, void* sk_dev,
                            void* evk_dev) {
  CHECK_CTX(x);
  if (!sk_dev || !evk_dev || n_steps < 0 || (n_steps && !steps)) return set_err(SECPE_EINVAL, "bad keygen arguments");
  Ctx& c = x->c;
  const int N = c.N, nm = c.n_mod, nq = c.n_q;
  double* sk = (double*)sk_dev;
  double* evk = (double*)evk_dev;
  const size_t key_doubles = c.key_bytes() / sizeof(double);
  std::vector<uint64_t> gal(1 + n_steps, 0);
  for (int i = 0; i < n_steps; ++i) gal[1 + i] = c.galois(steps[i]);
  auto fn = [&](Builder& b) {
    std::vector<SampleJob> js{c.secret_h > 0 ? SampleJob{sk, seed, (1ull << 56), nm, nq, SAMPLE_SPARSE, c.secret_h}
                                             : SampleJob{sk, seed, (1ull << 56), nm, nq, SAMPLE_TERNARY, 0}};
    b.sample(js);
    b.ntt({NttJob{sk, sk, nm, nq, 0, 0}}, false);
    double* s2 = b.scratch((size_t)nm * N);
    double* sp = b.scratch((size_t)nm * N);
    double* e = b.scratch((size_t)nm * N);
    EwJob sq{};
    sq.o0 = s2; sq.a0 = sk; sq.b0 = sk; sq.n_limbs = nm; sq.n_chain = nq; sq.op = EW_MUL;
    b.ew({sq});
    for (int kk = 0; kk <= n_steps; ++kk) {
      double* key = evk + (size_t)kk * key_doubles;
      const uint64_t purpose = kk == 0 ? 2 : 3;
      const uint64_t obj = kk == 0 ? 0 : gal[kk];
      const double* sfrom = s2;
      if (kk > 0) {
        b.automorph({AutoJob{sk, sp, nm, nq, (uint32_t)gal[kk], 0}});
        sfrom = sp;
      }
      for (int j = 0; j < c.dnum; ++j) {
        double* kb = key + (size_t)(2 * j) * nm * N;
        double* ka = key + (size_t)(2 * j + 1) * nm * N;
        const uint64_t tag = (purpose << 56) | ((obj & 0xFFFFFFFFull) << 24) | ((uint64_t)(j & 0xFFF) << 12);
        b.sample({SampleJob{ka, seed, tag, nm, nq, SAMPLE_UNIFORM, 0}, SampleJob{e, seed, tag, nm, nq, SAMPLE_CBD, 0}});
        b.ntt({NttJob{ka, ka, nm, nq, 0, 0}, NttJob{e, e, nm, nq, 0, 0}}, false);
        std::vector<double> kv(nm, 0.0);
        // the gadget P * T_j: T_j = 1 on the chain primes of digit j, 0 elsewhere
        for (int t = 0; t < nq; ++t) {
          if (t / c.alpha != j) continue;
          uint64_t P = 1;
          for (int k = 0; k < c.n_p; ++k) P = hmul(P, c.mod[nq + k] % c.mod[t], c.mod[t]);
          kv[t] = (double)P;
        }
        EwJob w{};
        w.o0 = kb; w.a1 = e; w.b0 = ka; w.b1 = sk; w.c0 = sfrom; w.k = b.put(kv);
        w.n_limbs = nm; w.n_chain = nq; w.op = EW_KEYB;
        b.ew({w});
      }
    }
  };
  int rc = run_client(x, fn);
  if (rc) return rc;
  rc = sync(c);
  if (rc) return rc;
  drop_graphs(c);
  c.keys.clear();
  c.keys_perm.clear();
  x->key_list.clear();
  x->evk = evk;
  for (int kk = 0; kk <= n_steps; ++kk) {
    const double* key = evk + (size_t)kk * key_doubles;
    x->key_list.push_back(key);
    if (kk == 0) c.keys[0] = key;
    else if (gal[kk] != 1 && !c.keys.count(gal[kk])) c.keys[gal[kk]] = key;
  }
  return 0;
}

extern "C" int secpe_keys_share(secpe_ctx* dst, const secpe_ctx* src) {
  CHECK_CTX(dst);
  if (!src || src == dst) return set_err(SECPE_EINVAL, "bad key source");
  const Ctx& a = src->c;
  Ctx& b = dst->c;
  if (a.mod != b.mod || a.N != b.N || a.n_q != b.n_q || a.dnum != b.dnum || a.device != b.device)
    return set_err(SECPE_EINVAL, "key source has other parameters or another device");
  if (a.keys.empty()) return set_err(SECPE_EINVAL, "key source has no keys");
  drop_graphs(b);
  b.keys = a.keys;
  b.keys_perm.clear();
  dst->evk = src->evk;
  dst->key_list = src->key_list;
  return 0;
}

extern "C" int secpe_key_owner_create(const secpe_ctx* x, const void* sk_dev, secpe_key_owner** out) {
  CHECK_CTX(x);
  if (!sk_dev || !out) return set_err(SECPE_EINVAL, "null argument");
  secpe_key_owner* o = new secpe_key_owner();
  o->sk = (const double*)sk_dev;
  o->device = x->c.device;
  o->mod = x->c.mod;
  *out = o;
  return 0;
}

extern "C" void secpe_key_owner_destroy(secpe_key_owner* o) { delete o; }

// ---------------------------------------------------------------------------
// client encryption / decryption
// ---------------------------------------------------------------------------
static int encrypt_impl(secpe_ctx* x, const void* sk_dev, const std::vector<double>& z, const int64_t* m_host,
                        double scale, uint64_t seed, secpe_ct* out) {
  Ctx& c = x->c;
  const int N = c.N;
  if (!sk_dev || !out || !out->data) return set_err(SECPE_EINVAL, "null buffer");
  CT o;
  o.d = (double*)out->data;
  o.level = c.n_q - 1;
  o.scale = scale;
  auto fn = [&](Builder& b) {
    int64_t* m = (int64_t*)b.scratch(N);
    if (m_host) {
      // the integer plaintext is uploaded through the descriptor arena
      const int64_t* src = (const int64_t*)b.put_bytes(m_host, sizeof(int64_t) * N);
      std::vector<const int64_t*> ms{src};
      b.encrypt_into(ms, {seed}, 4, {0}, (const double*)sk_dev, {o});
    } else {
      EncodeJob ej{};
      ej.z = b.put(z);
      ej.m = m;
      ej.scale_hi = scale * 2.0 / (double)N;
      ej.scale_lo = 0.0;
      ej.nnz = (int)z.size();
      b.encode({ej});
      b.encrypt_into({m}, {seed}, 4, {0}, (const double*)sk_dev, {o});
    }
  };
  int rc = run_client(x, fn);
  if (rc) return rc;
  out->level = o.level;
  out->scale = o.scale;
  return 0;
}

extern "C" int secpe_encrypt(secpe_ctx* x, const void* sk_dev, const double* logits, int K, int C, uint64_t seed,
                             secpe_ct* out) {
  CHECK_CTX(x);
  if (!logits || K < 1 || C < 1) return set_err(SECPE_EINVAL, "bad logits");
  const int cp = 1 << ilog2_ceil(C), kp = 1 << ilog2_ceil(K);
  if ((int64_t)cp * kp > x->c.N / 2) return set_err(SECPE_EINVAL, "K' * C' exceeds the slot count");
  std::vector<double> z((size_t)kp * cp, 0.0);
  for (int k = 0; k < K; ++k)
    for (int j = 0; j < C; ++j) z[(size_t)k * cp + j] = logits[(size_t)k * C + j];
  return encrypt_impl(x, sk_dev, z, nullptr, ldexp(1.0, x->c.log_scale), seed, out);
}

extern "C" int secpe_encrypt_coeffs(secpe_ctx* x, const void* sk_dev, const int64_t* m, double scale, uint64_t seed,
                                    secpe_ct* out) {
  CHECK_CTX(x);
  if (!m) return set_err(SECPE_EINVAL, "null plaintext");
  return encrypt_impl(x, sk_dev, {}, m, scale, seed, out);
}

static int decrypt_to_device(secpe_ctx* x, const void* sk_dev, const secpe_ct* ct, int nslots, int64_t** m_dev,
                             double** z_dev) {
  Ctx& c = x->c;
  const int N = c.N;
  if (!sk_dev || !ct || !ct->data) return set_err(SECPE_EINVAL, "null buffer");
  if (ct->level < 1 || ct->level >= c.n_q) return set_err(SECPE_EINVAL, "decryption needs a level in [1, n_q)");
  CT in;
  in.d = (double*)ct->data;
  in.level = ct->level;
  in.scale = ct->scale;
  auto fn = [&](Builder& b) {
    double* r = b.scratch(2 * (size_t)N);
    int64_t* m = (int64_t*)b.scratch(N);
    double* z = b.scratch(std::max(nslots, 1));
    EwJob d{};
    d.o0 = r; d.a0 = b.c0(in); d.a1 = b.c1(in); d.b0 = (const double*)sk_dev;
    d.n_limbs = 2; d.n_chain = 2; d.op = EW_DEC2;
    b.ew({d});
    b.ntt({NttJob{r, r, 2, 2, 0, 0}}, true);
    b.lift({LiftJob{r, r + N, r, m, 0, 0}});
    if (nslots > 0) b.decode(m, z, nslots, 1.0 / in.scale);
    *m_dev = m;
    *z_dev = z;
  };
  return run_client(x, fn);
}

extern "C" int secpe_decrypt(secpe_ctx* x, const void* sk_dev, const secpe_ct* ct, int nslots, double* z_out,
                             int* argmax_out) {
  CHECK_CTX(x);
  if (nslots < 1 || nslots > x->c.N / 2 || !z_out) return set_err(SECPE_EINVAL, "bad slot count");
  int64_t* m = nullptr;
  double* z = nullptr;
  int rc = decrypt_to_device(x, sk_dev, ct, nslots, &m, &z);
  if (rc) return rc;
  hipError_t e = hipMemcpyAsync(z_out, z, sizeof(double) * nslots, hipMemcpyDeviceToHost, x->c.stream);
  if (e != hipSuccess) return hip_fail("hipMemcpyAsync", e);
  rc = sync(x->c);
  if (rc) return rc;
  if (argmax_out) {
    int best = 0;
    for (int j = 1; j < nslots; ++j)
      if (z_out[j] > z_out[best]) best = j;
    *argmax_out = best;
  }
  return 0;
}

extern "C" int secpe_decrypt_coeffs(secpe_ctx* x, const void* sk_dev, const secpe_ct* ct, int64_t* m_out) {
  CHECK_CTX(x);
  if (!m_out) return set_err(SECPE_EINVAL, "null output");
  int64_t* m = nullptr;
  double* z = nullptr;
  int rc = decrypt_to_device(x, sk_dev, ct, 0, &m, &z);
  if (rc) return rc;
  hipError_t e = hipMemcpyAsync(m_out, m, sizeof(int64_t) * x->c.N, hipMemcpyDeviceToHost, x->c.stream);
  if (e != hipSuccess) return hip_fail("hipMemcpyAsync", e);
  return sync(x->c);
}

// ---------------------------------------------------------------------------
// evaluation
// ---------------------------------------------------------------------------
static std::vector<ArgmaxQuery> make_queries(secpe_ctx* x, int n, const secpe_ct* in, const int* K, const int* C,
                                             const double* dmin, const double* dmax, const uint64_t* rs,
                                             secpe_ct* out) {
  std::vector<ArgmaxQuery> q(n);
  for (int i = 0; i < n; ++i) {
    q[i].in.d = (double*)in[i].data;
    q[i].in.level = in[i].level;
    q[i].in.scale = in[i].scale;
    q[i].K = K[i];
    q[i].C = C[i];
    q[i].d_min = dmin[i];
    q[i].d_max = dmax[i];
    q[i].refresh_seed = rs[i];
    q[i].out.d = out ? (double*)out[i].data : nullptr;
  }
  (void)x;
  return q;
}

// packed queries: n_b[i] blocks for ciphertext i, their K, C, bounds concatenated
static int make_packed(secpe_ctx* x, int n, const secpe_ct* in, const int* n_b, const int* K, const int* C,
                       const double* dmin, const double* dmax, const uint64_t* rs, secpe_ct* out,
                       std::vector<ArgmaxQuery>& q) {
  q.assign(n, ArgmaxQuery{});
  size_t off = 0;
  for (int i = 0; i < n; ++i) {
    if (!in[i].data) return set_err(SECPE_EINVAL, "null input ciphertext");
    if (in[i].level < 0 || in[i].level >= x->c.n_q) return set_err(SECPE_EINVAL, "input level out of range");
    if (n_b[i] < 1) return set_err(SECPE_EINVAL, "a packed ciphertext needs at least one block");
    ArgmaxQuery& a = q[i];
    for (int j = 0; j < n_b[i]; ++j, ++off) {
      if (K[off] < 1 || C[off] < 1) return set_err(SECPE_EINVAL, "K and C must be positive");
      if (!(dmax[off] > dmin[off])) return set_err(SECPE_EINVAL, "need d_max > d_min");
      a.bK.push_back(K[off]);
      a.bC.push_back(C[off]);
      a.blo.push_back(dmin[off]);
      a.bhi.push_back(dmax[off]);
    }
    int kp, cp, bsz;
    packed_shape(a.bK, a.bC, &kp, &cp, &bsz);
    if ((int64_t)n_b[i] * bsz > x->c.N / 2) return set_err(SECPE_EINVAL, "packed queries exceed the slot count");
    a.in.d = (double*)in[i].data;
    a.in.level = in[i].level;
    a.in.scale = in[i].scale;
    a.K = kp;
    a.C = cp;
    a.d_min = a.blo[0];
    a.d_max = a.bhi[0];
    a.refresh_seed = rs[i];
    a.out.d = out ? (double*)out[i].data : nullptr;
  }
  return 0;
}

extern "C" int secpe_packed_shape(secpe_ctx* x, int n, const int* K, const int* C, int* out3) {
  CHECK_CTX(x);
  if (n < 1 || !K || !C || !out3) return set_err(SECPE_EINVAL, "bad arguments");
  for (int i = 0; i < n; ++i)
    if (K[i] < 1 || C[i] < 1) return set_err(SECPE_EINVAL, "K and C must be positive");
  std::vector<int> k(K, K + n), c(C, C + n);
  packed_shape(k, c, &out3[0], &out3[1], &out3[2]);
  const int per = (x->c.N / 2) / out3[2];
  if (per < 1) return set_err(SECPE_EINVAL, "one block exceeds the slot count");
  return per;
}

extern "C" int secpe_encrypt_packed(secpe_ctx* x, const void* sk_dev, int n, const double* logits, const int* K,
                                    const int* C, uint64_t seed, secpe_ct* out) {
  CHECK_CTX(x);
  int shape[3];
  const int per = secpe_packed_shape(x, n, K, C, shape);
  if (per < 0) return per;
  if (n > per) return set_err(SECPE_EINVAL, "packed queries exceed the slot count");
  if (!logits) return set_err(SECPE_EINVAL, "null logits");
  const int cp = shape[1], bsz = shape[2];
  std::vector<double> z((size_t)n * bsz, 0.0);
  const double* y = logits;
  for (int b = 0; b < n; ++b) {
    for (int k = 0; k < K[b]; ++k)
      for (int j = 0; j < C[b]; ++j) z[(size_t)b * bsz + (size_t)k * cp + j] = y[(size_t)k * C[b] + j];
    y += (size_t)K[b] * C[b];
  }
  return encrypt_impl(x, sk_dev, z, nullptr, ldexp(1.0, x->c.log_scale), seed, out);
}

extern "C" size_t secpe_packed_workspace_bytes(secpe_ctx* x, int n, const int* n_b, const int* K, const int* C) {
  if (!x || n < 1 || !n_b || !K || !C) return 0;
  Ctx& c = x->c;
  size_t tot = 0;
  for (int i = 0; i < n; ++i) tot += (size_t)std::max(0, n_b[i]);
  std::vector<secpe_ct> in(n), out(n);
  std::vector<double> dmin(tot, -1.0), dmax(tot, 1.0);
  std::vector<uint64_t> rs(n, 0);
  for (int i = 0; i < n; ++i) {
    in[i].data = (void*)(uintptr_t)0x200000000000ull;
    in[i].level = c.n_q - 1;
    in[i].scale = ldexp(1.0, c.log_scale);
    out[i].data = (void*)(uintptr_t)0x300000000000ull;
  }
  std::vector<ArgmaxQuery> q;
  if (make_packed(x, n, in.data(), n_b, K, C, dmin.data(), dmax.data(), rs.data(), out.data(), q)) return 0;
  Builder dry(c, (char*)(uintptr_t)0x100000000000ull, (size_t)1 << 44, (char*)(uintptr_t)0x400000000000ull,
              (size_t)1 << 40, true);
  build_argmax(dry, q);
  if (dry.err_code) {
    set_err(dry.err_code, dry.err);
    return 0;
  }
  return dry.need_bytes() + 4096;
}

extern "C" int secpe_eval_argmax_packed(secpe_ctx* x, const secpe_key_owner* owner, int n, const secpe_ct* in,
                                        const int* n_b, const int* K, const int* C, const double* dmin,
                                        const double* dmax, const uint64_t* rs, void* ws, size_t ws_bytes,
                                        secpe_ct* out) {
  CHECK_CTX(x);
  if (n < 1 || !in || !n_b || !K || !C || !dmin || !dmax || !rs || !ws || !out)
    return set_err(SECPE_EINVAL, "null argument");
  for (int i = 0; i < n; ++i)
    if (!out[i].data) return set_err(SECPE_EINVAL, "null output ciphertext");
  const double* rsk = nullptr;
  int rc = owner_sk(x, owner, &rsk);
  if (rc) return rc;
  std::vector<ArgmaxQuery> q;
  rc = make_packed(x, n, in, n_b, K, C, dmin, dmax, rs, out, q);
  if (rc) return rc;
  rc = run_build(x, (char*)ws, ws_bytes, [&](Builder& b) { b.refresh_sk = rsk; build_argmax(b, q); });
  if (rc) return rc;
  for (int i = 0; i < n; ++i) { out[i].level = q[i].out.level; out[i].scale = q[i].out.scale; }
  return 0;
}

static void phoenix_query(secpe_ctx* x, const secpe_ct* in, int K, int C, double dmin, double dmax, uint64_t rs,
                          secpe_ct* out, ArgmaxQuery& q) {
  (void)x;
  q.in.d = (double*)in->data;
  q.in.level = in->level;
  q.in.scale = in->scale;
  q.K = K;
  q.C = C;
  q.d_min = dmin;
  q.d_max = dmax;
  q.refresh_seed = rs;
  q.out.d = (double*)out->data;
}

extern "C" size_t secpe_phoenix_workspace_bytes(secpe_ctx* x, int K, int C) {
  if (!x || K < 1 || C < 2) return 0;
  Ctx& c = x->c;
  secpe_ct in{(void*)(uintptr_t)0x200000000000ull, c.n_q - 1, ldexp(1.0, c.log_scale)};
  secpe_ct out{(void*)(uintptr_t)0x300000000000ull, 0, 0.0};
  ArgmaxQuery q;
  phoenix_query(x, &in, K, C, -1.0, 1.0, 0, &out, q);
  Builder dry(c, (char*)(uintptr_t)0x100000000000ull, (size_t)1 << 44, (char*)(uintptr_t)0x400000000000ull,
              (size_t)1 << 40, true);
  build_phoenix(dry, q);
  if (dry.err_code) {
    set_err(dry.err_code, dry.err);
    return 0;
  }
  return dry.need_bytes() + 4096;
}

extern "C" int secpe_eval_argmax_phoenix(secpe_ctx* x, const secpe_key_owner* owner, const secpe_ct* in, int K, int C,
                                         double dmin, double dmax, uint64_t rs, void* ws, size_t ws_bytes,
                                         secpe_ct* out) {
  CHECK_CTX(x);
  if (!in || !in->data || !out || !out->data || !ws) return set_err(SECPE_EINVAL, "null argument");
  if (in->level < 0 || in->level >= x->c.n_q) return set_err(SECPE_EINVAL, "input level out of range");
  if (K < 1 || C < 2) return set_err(SECPE_EINVAL, "need K >= 1 and C >= 2");
  if (!(dmax > dmin)) return set_err(SECPE_EINVAL, "need d_max > d_min");
  const double* rsk = nullptr;
  int rc = owner_sk(x, owner, &rsk);
  if (rc) return rc;
  ArgmaxQuery q;
  phoenix_query(x, in, K, C, dmin, dmax, rs, out, q);
  rc = run_build(x, (char*)ws, ws_bytes, [&](Builder& b) { b.refresh_sk = rsk; build_phoenix(b, q); });
  if (rc) return rc;
  out->level = q.out.level;
  out->scale = q.out.scale;
  return 0;
}

static int check_queries(secpe_ctx* x, int n, const secpe_ct* in, const int* K, const int* C, const double* dmin,
                         const double* dmax) {
  for (int i = 0; i < n; ++i) {
    if (!in[i].data) return set_err(SECPE_EINVAL, "null input ciphertext");
    if (in[i].level < 0 || in[i].level >= x->c.n_q) return set_err(SECPE_EINVAL, "input level out of range");
    if (K[i] < 1 || C[i] < 1) return set_err(SECPE_EINVAL, "K and C must be positive");
    const int cp = 1 << ilog2_ceil(C[i]), kp = 1 << ilog2_ceil(K[i]);
    if ((int64_t)cp * kp > x->c.N / 2) return set_err(SECPE_EINVAL, "K' * C' exceeds the slot count");
    if (!(dmax[i] > dmin[i])) return set_err(SECPE_EINVAL, "need d_max > d_min");
  }
  return 0;
}

extern "C" size_t secpe_workspace_bytes(secpe_ctx* x, int n, const int* K, const int* C) {
  if (!x || n < 1 || !K || !C) return 0;
  std::vector<secpe_ct> in(n), out(n);
  std::vector<double> dmin(n, -1.0), dmax(n, 1.0);
  std::vector<uint64_t> rs(n, 0);
  Ctx& c = x->c;
  for (int i = 0; i < n; ++i) {
    in[i].data = (void*)(uintptr_t)0x200000000000ull;
    in[i].level = c.n_q - 1;
    in[i].scale = ldexp(1.0, c.log_scale);
    out[i].data = (void*)(uintptr_t)0x300000000000ull;
  }
  if (check_queries(x, n, in.data(), K, C, dmin.data(), dmax.data())) return 0;
  std::vector<ArgmaxQuery> q = make_queries(x, n, in.data(), K, C, dmin.data(), dmax.data(), rs.data(), out.data());
  Builder dry(c, (char*)(uintptr_t)0x100000000000ull, (size_t)1 << 44, (char*)(uintptr_t)0x400000000000ull, (size_t)1 << 40, true);
  build_argmax(dry, q);
  if (dry.err_code) {
    set_err(dry.err_code, dry.err);
    return 0;
  }
  return dry.need_bytes() + 4096;
}

static uint64_t fnv(uint64_t h, const void* p, size_t n) {
  const unsigned char* b = (const unsigned char*)p;
  for (size_t i = 0; i < n; ++i) { h ^= b[i]; h *= 1099511628211ull; }
  return h;
}

extern "C" int secpe_eval_argmax_batch(secpe_ctx* x, const secpe_key_owner* owner, int n, const secpe_ct* in,
                                       const int* K, const int* C, const double* dmin, const double* dmax,
                                       const uint64_t* rs, void* ws, size_t ws_bytes, secpe_ct* out, int flags) {
  CHECK_CTX(x);
  if (n < 1 || !in || !K || !C || !dmin || !dmax || !rs || !ws || !out) return set_err(SECPE_EINVAL, "null argument");
  const double* rsk = nullptr;
  int rc = owner_sk(x, owner, &rsk);
  if (rc) return rc;
  rc = check_queries(x, n, in, K, C, dmin, dmax);
  if (rc) return rc;
  for (int i = 0; i < n; ++i)
    if (!out[i].data) return set_err(SECPE_EINVAL, "null output ciphertext");
  Ctx& c = x->c;
  std::vector<ArgmaxQuery> q = make_queries(x, n, in, K, C, dmin, dmax, rs, out);
  if (!(flags & SECPE_GRAPH)) {
    rc = run_build(x, (char*)ws, ws_bytes, [&](Builder& b) { b.refresh_sk = rsk; build_argmax(b, q); });
    if (rc) return rc;
    for (int i = 0; i < n; ++i) { out[i].level = q[i].out.level; out[i].scale = q[i].out.scale; }
    return 0;
  }
  // graph mode: one captured graph per distinct argument set
  uint64_t h = 1469598103934665603ull;
  h = fnv(h, &n, sizeof(n));
  for (int i = 0; i < n; ++i) {
    h = fnv(h, &in[i], sizeof(secpe_ct));
    h = fnv(h, &out[i].data, sizeof(void*));
    h = fnv(h, &K[i], sizeof(int));
    h = fnv(h, &C[i], sizeof(int));
    h = fnv(h, &dmin[i], sizeof(double));
    h = fnv(h, &dmax[i], sizeof(double));
    h = fnv(h, &rs[i], sizeof(uint64_t));
  }
  h = fnv(h, &ws, sizeof(ws));
  h = fnv(h, &ws_bytes, sizeof(ws_bytes));
  h = fnv(h, &rsk, sizeof(rsk));
  for (GraphEntry& g : c.graphs) {
    if (g.hash != h) continue;
    hipError_t e = hipGraphLaunch(g.exec, c.stream);
    if (e != hipSuccess) return hip_fail("hipGraphLaunch", e);
    for (int i = 0; i < n; ++i) { out[i].level = g.out_level[i]; out[i].scale = g.out_scale[i]; }
    memcpy(c.counters, g.counters, sizeof(c.counters));
    c.ks_alg_limbs = g.ks_alg_limbs;
    return 0;
  }
  if (!c.stream) return set_err(SECPE_EINVAL, "graph capture needs a non-null stream");
  GraphEntry g;
  g.hash = h;
  // size the graph's own descriptor arena with a dry run
  {
    Builder dry(c, (char*)ws, ws_bytes, (char*)(uintptr_t)0x400000000000ull, (size_t)1 << 40, true);
    dry.refresh_sk = rsk;
    std::vector<ArgmaxQuery> qd = q;
    build_argmax(dry, qd);
    if (dry.err_code) return set_err(dry.err_code, dry.err);
    g.arena_bytes = dry.blob_bytes() + 4096;
  }
  hipError_t e = hipMalloc((void**)&g.arena, g.arena_bytes);
  if (e != hipSuccess) return hip_fail("hipMalloc", e);
  Builder b(c, (char*)ws, ws_bytes, g.arena, g.arena_bytes, false);
  b.refresh_sk = rsk;
  build_argmax(b, q);
  if (b.err_code) { (void)hipFree(g.arena); return set_err(b.err_code, b.err); }
  e = hipMemcpy(g.arena, b.blob_.data(), b.blob_.size(), hipMemcpyHostToDevice);
  if (e != hipSuccess) { (void)hipFree(g.arena); return hip_fail("hipMemcpy", e); }
  e = hipStreamBeginCapture(c.stream, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) { (void)hipFree(g.arena); return hip_fail("hipStreamBeginCapture", e); }
  launch_cmds(c, b.cmds_, g.arena);
  e = hipStreamEndCapture(c.stream, &g.graph);
  if (e != hipSuccess) { (void)hipFree(g.arena); return hip_fail("hipStreamEndCapture", e); }
  e = hipGraphInstantiate(&g.exec, g.graph, nullptr, nullptr, 0);
  if (e != hipSuccess) { (void)hipGraphDestroy(g.graph); (void)hipFree(g.arena); return hip_fail("hipGraphInstantiate", e); }
  for (int i = 0; i < n; ++i) { g.out_level.push_back(q[i].out.level); g.out_scale.push_back(q[i].out.scale); }
  memcpy(g.counters, b.counters, sizeof(g.counters));
  g.ks_alg_limbs = b.ks_alg_limbs;
  c.graphs.push_back(g);
  e = hipGraphLaunch(g.exec, c.stream);
  if (e != hipSuccess) return hip_fail("hipGraphLaunch", e);
  for (int i = 0; i < n; ++i) { out[i].level = g.out_level[i]; out[i].scale = g.out_scale[i]; }
  memcpy(c.counters, g.counters, sizeof(c.counters));
  c.ks_alg_limbs = g.ks_alg_limbs;
  return 0;
}

extern "C" int secpe_eval_argmax(secpe_ctx* x, const secpe_key_owner* owner, const secpe_ct* in, int K, int C,
                                 double d_min, double d_max, uint64_t refresh_seed, void* ws, size_t ws_bytes,
                                 secpe_ct* out) {
  return secpe_eval_argmax_batch(x, owner, 1, in, &K, &C, &d_min, &d_max, &refresh_seed, ws, ws_bytes, out, 0);
}

static size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

extern "C" int secpe_eval_argmax_noalloc(secpe_ctx* x, const secpe_key_owner* owner, const secpe_ct* in, int K, int C,
                                         double d_min, double d_max, uint64_t refresh_seed, secpe_ct* out) {
  CHECK_CTX(x);
  if (!in || !out || !out->data) return set_err(SECPE_EINVAL, "null argument");
  const double* rsk = nullptr;
  int rc = owner_sk(x, owner, &rsk);
  if (rc) return rc;
  rc = check_queries(x, 1, in, &K, &C, &d_min, &d_max);
  if (rc) return rc;
  Ctx& c = x->c;
  char* base = scratch_ptr(c.device);
  if (!base) return set_err(SECPE_EDEVICE, "no scratch address for this device");
  std::vector<ArgmaxQuery> q = make_queries(x, 1, in, &K, &C, &d_min, &d_max, &refresh_seed, out);
  // size the workspace and the descriptor blob with a dry run (host only)
  size_t blob = 0, need = 0;
  {
    Builder dry(c, (char*)(uintptr_t)0x100000000000ull, (size_t)1 << 44, (char*)(uintptr_t)0x400000000000ull,
                (size_t)1 << 40, true);
    dry.refresh_sk = rsk;
    std::vector<ArgmaxQuery> qd = q;
    build_argmax(dry, qd);
    if (dry.err_code) return set_err(dry.err_code, dry.err);
    blob = dry.blob_bytes();
    need = dry.need_bytes();
  }
  const size_t arena_bytes = align256(blob + 1);
  if (blob > c.staging_bytes || blob > SECPE_NOALLOC_BLOB_BYTES)
    return set_err(SECPE_ENOMEM, "descriptor blob of " + std::to_string(blob) + " bytes exceeds the no-allocation limit of " +
                                     std::to_string((size_t)SECPE_NOALLOC_BLOB_BYTES));
  if (arena_bytes + need > SECPE_NOALLOC_SCRATCH_BYTES)
    return set_err(SECPE_ENOMEM, "evaluation needs " + std::to_string(arena_bytes + need) +
                                     " bytes of scratch; the no-allocation scratch holds " +
                                     std::to_string((size_t)SECPE_NOALLOC_SCRATCH_BYTES));
  // layout of the scratch: descriptor arena, then the workspace
  Builder b(c, base + arena_bytes, SECPE_NOALLOC_SCRATCH_BYTES - arena_bytes, base, arena_bytes, false);
  b.refresh_sk = rsk;
  build_argmax(b, q);
  if (b.err_code) return set_err(b.err_code, b.err);
  if (b.arena_overflow()) return set_err(SECPE_ENOMEM, "descriptor arena overflow");
  rc = submit(c, b, base, arena_bytes, false);
  if (rc) return set_err(rc == -2 ? SECPE_ENOMEM : SECPE_EDEVICE, "kernel submission failed");
  memcpy(c.counters, b.counters, sizeof(c.counters));
  c.ks_alg_limbs = b.ks_alg_limbs;
  out->level = q[0].out.level;
  out->scale = q[0].out.scale;
  return 0;
}

extern "C" int secpe_counters(const secpe_ctx* x, int64_t* out8) {
  CHECK_CTX(x);
  memcpy(out8, x->c.counters, sizeof(int64_t) * 8);
  return 0;
}

extern "C" int secpe_keyswitch_traffic(const secpe_ctx* x, int64_t* alg_bytes) {
  CHECK_CTX(x);
  if (!alg_bytes) return set_err(SECPE_EINVAL, "null argument");
  *alg_bytes = x->c.ks_alg_limbs * (int64_t)x->c.limb_bytes();
  return 0;
}

extern "C" int secpe_sync(secpe_ctx* x) {
  CHECK_CTX(x);
  return sync(x->c);
}

// ---------------------------------------------------------------------------
// export / import
// ---------------------------------------------------------------------------
static int download_limbs(secpe_ctx* x, const double* dev, size_t n, uint64_t* host) {
  std::vector<double> tmp(n);
  hipError_t e = hipMemcpyAsync(tmp.data(), dev, n * sizeof(double), hipMemcpyDeviceToHost, x->c.stream);
  if (e != hipSuccess) return hip_fail("hipMemcpyAsync", e);
  int rc = sync(x->c);
  if (rc) return rc;
  for (size_t i = 0; i < n; ++i) host[i] = (uint64_t)tmp[i];
  return 0;
}

extern "C" int secpe_ct_export(secpe_ctx* x, const secpe_ct* ct, uint64_t* host_out) {
  CHECK_CTX(x);
  if (!ct || !ct->data || !host_out || ct->level < 0 || ct->level >= x->c.n_q) return set_err(SECPE_EINVAL, "bad ciphertext");
  Ctx& c = x->c;
  const int N = c.N, nl = ct->level + 1;
  double* out = nullptr;
  auto fn = [&](Builder& b) {
    out = b.scratch(2 * (size_t)nl * N);
    const double* d = (const double*)ct->data;
    b.ntt({NttJob{d, out, nl, nl, 0, 0}, NttJob{d + (size_t)c.n_q * N, out + (size_t)nl * N, nl, nl, 0, 0}}, true);
  };
  int rc = run_client(x, fn);
  if (rc) return rc;
  return download_limbs(x, out, 2 * (size_t)nl * N, host_out);
}

extern "C" int secpe_ct_import(secpe_ctx* x, const uint64_t* host_in, int level, double scale, secpe_ct* out) {
  CHECK_CTX(x);
  Ctx& c = x->c;
  if (!host_in || !out || !out->data || level < 0 || level >= c.n_q) return set_err(SECPE_EINVAL, "bad import");
  const int N = c.N, nl = level + 1;
  std::vector<double> tmp(2 * (size_t)nl * N);
  for (int p = 0; p < 2; ++p)
    for (int l = 0; l < nl; ++l)
      for (int k = 0; k < N; ++k) {
        const uint64_t v = host_in[((size_t)p * nl + l) * N + k];
        if (v >= c.mod[l]) return set_err(SECPE_EINVAL, "residue not canonical");
        tmp[((size_t)p * nl + l) * N + k] = (double)v;
      }
  double* d = (double*)out->data;
  double* stage = nullptr;
  auto fn = [&](Builder& b) {
    stage = b.scratch(tmp.size());
    b.ntt({NttJob{stage, d, nl, nl, 0, 0}, NttJob{stage + (size_t)nl * N, d + (size_t)c.n_q * N, nl, nl, 0, 0}}, false);
  };
  // size the scratch, upload, then transform
  Builder dry(c, (char*)(uintptr_t)0x100000000000ull, (size_t)1 << 44, (char*)(uintptr_t)0x400000000000ull, (size_t)1 << 40, true);
  fn(dry);
  int rc = ensure_buffer(c, &c.client, &c.client_bytes, dry.need_bytes() + 4096);
  if (rc) return rc;
  rc = sync(c);
  if (rc) return rc;
  Builder probe(c, c.client, c.client_bytes, (char*)(uintptr_t)0x400000000000ull, (size_t)1 << 40, true);
  fn(probe);
  hipError_t e = hipMemcpy(stage, tmp.data(), tmp.size() * sizeof(double), hipMemcpyHostToDevice);
  if (e != hipSuccess) return hip_fail("hipMemcpy", e);
  rc = run_build(x, c.client, c.client_bytes, fn, false);
  if (rc) return rc;
  out->level = level;
  out->scale = scale;
  return 0;
}

extern "C" int secpe_key_export(secpe_ctx* x, const void* evk_dev, int key, int digit, int which, int prime,
                                uint64_t* host_out) {
  CHECK_CTX(x);
  Ctx& c = x->c;
  if (!evk_dev || key < 0 || digit < 0 || digit >= c.dnum || which < 0 || which > 1 || prime < 0 || prime >= c.n_mod)
    return set_err(SECPE_EINVAL, "bad key index");
  const int N = c.N;
  const double* src = (const double*)evk_dev + (size_t)key * (c.key_bytes() / sizeof(double)) +
                      ((size_t)(2 * digit + which) * c.n_mod + prime) * N;
  double* out = nullptr;
  // a one-limb transform with the right prime: present it as limb 'prime' of a basis
  const int nch = prime < c.n_q ? prime + 1 : c.n_q;
  const int limb = prime < c.n_q ? prime : c.n_q + (prime - c.n_q);
  auto fn = [&](Builder& b) {
    out = b.scratch(N);
    b.ntt({NttJob{src - (size_t)limb * N, out - (size_t)limb * N, limb + 1, nch, 0, limb}}, true);
  };
  int rc = run_client(x, fn);
  if (rc) return rc;
  return download_limbs(x, out, N, host_out);
}

extern "C" int secpe_sk_export(secpe_ctx* x, const void* sk_dev, int64_t* host_out) {
  CHECK_CTX(x);
  Ctx& c = x->c;
  const int N = c.N;
  double* out = nullptr;
  auto fn = [&](Builder& b) {
    out = b.scratch(N);
    b.ntt({NttJob{(const double*)sk_dev, out, 1, 1, 0, 0}}, true);
  };
  int rc = run_client(x, fn);
  if (rc) return rc;
  std::vector<uint64_t> r(N);
  rc = download_limbs(x, out, N, r.data());
  if (rc) return rc;
  const uint64_t q = c.mod[0];
  for (int i = 0; i < N; ++i) host_out[i] = r[i] > q / 2 ? (int64_t)r[i] - (int64_t)q : (int64_t)r[i];
  return 0;
}

// ---------------------------------------------------------------------------
// primitive operations
// ---------------------------------------------------------------------------
static CT to_ct(const secpe_ct* a) {
  CT x;
  x.d = (double*)a->data;
  x.level = a->level;
  x.scale = a->scale;
  return x;
}

extern "C" size_t secpe_op_workspace_bytes(secpe_ctx* x) {
  if (!x) return 0;
  Ctx& c = x->c;
  // a few ciphertexts plus one key switch at the top level, plus a refresh
  const size_t limb = c.limb_bytes();
  const size_t ks = (size_t)(c.n_q + (size_t)c.dnum * (c.n_q + c.n_p) + 2 * (c.n_q + c.n_p) + 2 * c.n_q) * limb;
  return 24 * c.ct_bytes() + 2 * ks + 8 * c.n_q * limb + ((size_t)1 << 20);
}

// run a builder body whose result is one ciphertext copied into 'out'
template <class F>
static int op_to_out(secpe_ctx* x, void* ws, size_t ws_bytes, secpe_ct* out, F body) {
  Ctx& c = x->c;
  if (!out || !out->data) return set_err(SECPE_EINVAL, "null output");
  CT res;
  int rc = run_build(x, (char*)ws, ws_bytes, [&](Builder& b) {
    std::vector<CT> rv = body(b);
    if (b.err_code) return;
    if (rv.empty()) { b.fail(SECPE_EINVAL, "operation produced no result"); return; }
    CT r = rv[0];
    EwJob e{};
    e.o0 = (double*)out->data;
    e.o1 = (double*)out->data + (size_t)c.n_q * c.N;
    e.a0 = b.c0(r);
    e.a1 = b.c1(r);
    e.n_limbs = r.level + 1;
    e.n_chain = r.level + 1;
    e.op = EW_COPY;
    b.ew({e});
    res = r;
  });
  if (rc) return rc;
  out->level = res.level;
  out->scale = res.scale;
  return 0;
}

extern "C" int secpe_op_add(secpe_ctx* x, const secpe_ct* a, const secpe_ct* b2, secpe_ct* out) {
  CHECK_CTX(x);
  size_t ws = secpe_op_workspace_bytes(x);
  int rc = ensure_buffer(x->c, &x->c.client, &x->c.client_bytes, ws);
  if (rc) return rc;
  return op_to_out(x, x->c.client, x->c.client_bytes, out, [&](Builder& b) { return b.add({{to_ct(a), to_ct(b2)}}, false); });
}
extern "C" int secpe_op_sub(secpe_ctx* x, const secpe_ct* a, const secpe_ct* b2, secpe_ct* out) {
  CHECK_CTX(x);
  size_t ws = secpe_op_workspace_bytes(x);
  int rc = ensure_buffer(x->c, &x->c.client, &x->c.client_bytes, ws);
  if (rc) return rc;
  return op_to_out(x, x->c.client, x->c.client_bytes, out, [&](Builder& b) { return b.add({{to_ct(a), to_ct(b2)}}, true); });
}
extern "C" int secpe_op_add_const(secpe_ctx* x, const secpe_ct* a, double v, secpe_ct* out) {
  CHECK_CTX(x);
  size_t ws = secpe_op_workspace_bytes(x);
  int rc = ensure_buffer(x->c, &x->c.client, &x->c.client_bytes, ws);
  if (rc) return rc;
  return op_to_out(x, x->c.client, x->c.client_bytes, out, [&](Builder& b) { return b.add_const({to_ct(a)}, {v}); });
}
extern "C" int secpe_op_mul_const(secpe_ctx* x, const secpe_ct* a, double v, double target, void* ws, size_t wsb,
                                  secpe_ct* out) {
  CHECK_CTX(x);
  return op_to_out(x, ws, wsb, out, [&](Builder& b) { return b.mul_const({to_ct(a)}, {v}, {target}); });
}
extern "C" int secpe_op_lincomb(secpe_ctx* x, const secpe_ct* a, double va, const secpe_ct* b2, double vb,
                                double target, int rescale, void* ws, size_t wsb, secpe_ct* out) {
  CHECK_CTX(x);
  if (!a) return SECPE_EINVAL;
  return op_to_out(x, ws, wsb, out, [&](Builder& b) {
    Builder::LinItem t{};
    t.a = to_ct(a);
    t.va = va;
    if (b2) { t.b = to_ct(b2); t.vb = vb; t.has_b = true; }
    t.target = target;
    return b.lincomb({t}, rescale != 0);
  });
}
extern "C" int secpe_op_mul_plain(secpe_ctx* x, const secpe_ct* a, const double* v, int nslots, double target, void* ws,
                                  size_t wsb, secpe_ct* out) {
  CHECK_CTX(x);
  std::vector<double> z(v, v + nslots);
  return op_to_out(x, ws, wsb, out, [&](Builder& b) { return b.mul_plain({to_ct(a)}, {z}, {target}); });
}
extern "C" int secpe_op_rescale(secpe_ctx* x, const secpe_ct* a, void* ws, size_t wsb, secpe_ct* out) {
  CHECK_CTX(x);
  return op_to_out(x, ws, wsb, out, [&](Builder& b) {
    CT in = to_ct(a);
    CT o = b.new_ct(in.level, in.scale);
    EwJob e{};
    e.o0 = b.c0(o); e.o1 = b.c1(o); e.a0 = b.c0(in); e.a1 = b.c1(in);
    e.n_limbs = in.level + 1; e.n_chain = in.level + 1; e.op = EW_COPY;
    b.ew({e});
    std::vector<CT> v{o};
    b.rescale(v);
    return v;
  });
}
extern "C" int secpe_op_mul_relin(secpe_ctx* x, const secpe_ct* a, const secpe_ct* b2, void* ws, size_t wsb,
                                  secpe_ct* out) {
  CHECK_CTX(x);
  return op_to_out(x, ws, wsb, out, [&](Builder& b) { return b.mul_relin({{to_ct(a), to_ct(b2)}}, false); });
}
extern "C" int secpe_op_mul_relin_rescale(secpe_ctx* x, const secpe_ct* a, const secpe_ct* b2, void* ws, size_t wsb,
                                          secpe_ct* out) {
  CHECK_CTX(x);
  return op_to_out(x, ws, wsb, out, [&](Builder& b) { return b.mul_relin({{to_ct(a), to_ct(b2)}}, true); });
}
extern "C" int secpe_op_rotate(secpe_ctx* x, const secpe_ct* a, int64_t step, void* ws, size_t wsb, secpe_ct* out) {
  CHECK_CTX(x);
  return op_to_out(x, ws, wsb, out, [&](Builder& b) { return b.rotate({to_ct(a)}, {step}); });
}
extern "C" int secpe_op_refresh(secpe_ctx* x, const secpe_key_owner* owner, const secpe_ct* a, uint64_t seed,
                                uint64_t index, void* ws, size_t wsb, secpe_ct* out) {
  CHECK_CTX(x);
  const double* rsk = nullptr;
  int rc = owner_sk(x, owner, &rsk);
  if (rc) return rc;
  return op_to_out(x, ws, wsb, out, [&](Builder& b) {
    b.refresh_sk = rsk;
    return b.refresh({to_ct(a)}, {seed}, {index});
  });
}
extern "C" int secpe_op_eval_odd9(secpe_ctx* x, const secpe_ct* a, const double* coef5, double gain, double target,
                                  void* ws, size_t wsb, secpe_ct* out) {
  CHECK_CTX(x);
  if (!coef5) return set_err(SECPE_EINVAL, "null coefficients");
  return op_to_out(x, ws, wsb, out, [&](Builder& b) { return b.eval_odd9({to_ct(a)}, {coef5}, {gain}, {target}); });
}

extern "C" int secpe_op_key_switch(secpe_ctx* x, int key, const uint64_t* d_host, int level, void* ws, size_t wsb,
                                   uint64_t* u0_host, uint64_t* u1_host) {
  CHECK_CTX(x);
  Ctx& c = x->c;
  if (key < 0 || key >= (int)x->key_list.size()) return set_err(SECPE_ENOKEY, "no such key");
  if (level < 0 || level >= c.n_q || !d_host || !u0_host || !u1_host) return set_err(SECPE_EINVAL, "bad arguments");
  const int N = c.N, nl = level + 1;
  // stage d as a ciphertext (c0 = d, c1 = 0) through import, then switch c0
  std::vector<uint64_t> h(2 * (size_t)nl * N, 0);
  memcpy(h.data(), d_host, sizeof(uint64_t) * (size_t)nl * N);
  char* wsc = (char*)ws;
  if (wsb < 2 * c.ct_bytes()) return set_err(SECPE_ENOMEM, "workspace too small");
  secpe_ct din{wsc, 0, 1.0};
  int rc = secpe_ct_import(x, h.data(), level, 1.0, &din);
  if (rc) return rc;
  secpe_ct uo{wsc + c.ct_bytes(), level, 1.0};
  const double* kp = x->key_list[key];
  rc = run_build(x, wsc + 2 * c.ct_bytes(), wsb - 2 * c.ct_bytes(), [&](Builder& b) {
    CT dd = to_ct(&din);
    CT uu = to_ct(&uo);
    b.key_switch({Builder::KsItem{b.c0(dd), level, kp, nullptr, nullptr, b.c0(uu), b.c1(uu)}});
  });
  if (rc) return rc;
  std::vector<uint64_t> o(2 * (size_t)nl * N);
  rc = secpe_ct_export(x, &uo, o.data());
  if (rc) return rc;
  memcpy(u0_host, o.data(), sizeof(uint64_t) * (size_t)nl * N);
  memcpy(u1_host, o.data() + (size_t)nl * N, sizeof(uint64_t) * (size_t)nl * N);
  return 0;
}

extern "C" int secpe_op_ntt(secpe_ctx* x, int prime, const uint64_t* in_host, int n, uint64_t* out_fwd,
                            uint64_t* out_rt) {
  CHECK_CTX(x);
  Ctx& c = x->c;
  if (prime < 0 || prime >= c.n_mod || n < 1 || !in_host) return set_err(SECPE_EINVAL, "bad arguments");
  const int N = c.N;
  const int nch = prime < c.n_q ? prime + 1 : c.n_q;
  const int limb = prime;  // chain prime t sits at limb t; special prime n_q + k at limb n_q + k with n_chain = n_q
  std::vector<double> tmp((size_t)n * N);
  for (size_t i = 0; i < tmp.size(); ++i) tmp[i] = (double)in_host[i];
  double *buf = nullptr, *fw = nullptr;
  auto fn = [&](Builder& b) {
    buf = b.scratch((size_t)n * N);
    fw = b.scratch((size_t)n * N);
    std::vector<NttJob> f, r;
    for (int i = 0; i < n; ++i) {
      double* s = buf + (size_t)i * N;
      double* d = fw + (size_t)i * N;
      f.push_back(NttJob{s - (size_t)limb * N, d - (size_t)limb * N, limb + 1, nch, 0, limb});
      r.push_back(NttJob{d - (size_t)limb * N, s - (size_t)limb * N, limb + 1, nch, 0, limb});
    }
    b.ntt(f, false);
    b.ntt(r, true);
  };
  Builder dry(c, (char*)(uintptr_t)0x100000000000ull, (size_t)1 << 44, (char*)(uintptr_t)0x400000000000ull, (size_t)1 << 40, true);
  fn(dry);
  int rc = ensure_buffer(c, &c.client, &c.client_bytes, dry.need_bytes() + 4096);
  if (rc) return rc;
  rc = sync(c);
  if (rc) return rc;
  Builder probe(c, c.client, c.client_bytes, (char*)(uintptr_t)0x400000000000ull, (size_t)1 << 40, true);
  fn(probe);
  hipError_t e = hipMemcpy(buf, tmp.data(), tmp.size() * sizeof(double), hipMemcpyHostToDevice);
  if (e != hipSuccess) return hip_fail("hipMemcpy", e);
  rc = run_build(x, c.client, c.client_bytes, fn, false);
  if (rc) return rc;
  if (out_fwd) {
    rc = download_limbs(x, fw, (size_t)n * N, out_fwd);
    if (rc) return rc;
  }
  if (out_rt) return download_limbs(x, buf, (size_t)n * N, out_rt);
  return sync(c);
}

extern "C" int secpe_op_ring_mul(secpe_ctx* x, int prime, const uint64_t* a_host, const uint64_t* b_host,
                                 uint64_t* out_host) {
  CHECK_CTX(x);
  Ctx& c = x->c;
  if (prime < 0 || prime >= c.n_mod || !a_host || !b_host || !out_host) return set_err(SECPE_EINVAL, "bad arguments");
  const int N = c.N;
  const int nch = prime < c.n_q ? prime + 1 : c.n_q;
  const int limb = prime;
  std::vector<double> tmp(2 * (size_t)N);
  for (int i = 0; i < N; ++i) { tmp[i] = (double)a_host[i]; tmp[N + i] = (double)b_host[i]; }
  double* buf = nullptr;
  // the views below present limb 'limb' of a basis; the element-wise product
  // runs over limbs 0..limb of both views, which fn2 allocates in full
  auto fn2 = [&](Builder& b) {
    buf = b.scratch((size_t)(limb + 2) * N * 2);
    double* a = buf + (size_t)limb * N;              // limb 'limb' of view A
    double* bb = buf + (size_t)(2 * limb + 1) * N;   // limb 'limb' of view B
    double* va = a - (size_t)limb * N;
    double* vb = bb - (size_t)limb * N;
    b.ntt({NttJob{va, va, limb + 1, nch, 0, limb}, NttJob{vb, vb, limb + 1, nch, 0, limb}}, false);
    EwJob e{};
    e.o0 = va; e.a0 = va; e.b0 = vb;
    e.n_limbs = limb + 1; e.n_chain = nch; e.op = EW_MUL;
    b.ew({e});
    b.ntt({NttJob{va, va, limb + 1, nch, 0, limb}}, true);
  };
  Builder dry(c, (char*)(uintptr_t)0x100000000000ull, (size_t)1 << 44, (char*)(uintptr_t)0x400000000000ull, (size_t)1 << 40, true);
  fn2(dry);
  int rc = ensure_buffer(c, &c.client, &c.client_bytes, dry.need_bytes() + 4096);
  if (rc) return rc;
  rc = sync(c);
  if (rc) return rc;
  Builder probe(c, c.client, c.client_bytes, (char*)(uintptr_t)0x400000000000ull, (size_t)1 << 40, true);
  fn2(probe);
  double* a = buf + (size_t)limb * N;
  double* bb = buf + (size_t)(2 * limb + 1) * N;
  hipError_t e = hipMemcpy(a, tmp.data(), (size_t)N * sizeof(double), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(bb, tmp.data() + N, (size_t)N * sizeof(double), hipMemcpyHostToDevice);
  if (e != hipSuccess) return hip_fail("hipMemcpy", e);
  rc = run_build(x, c.client, c.client_bytes, fn2, false);
  if (rc) return rc;
  return download_limbs(x, a, N, out_host);
}

extern "C" int secpe_op_encode(secpe_ctx* x, const double* z, int nslots, double scale, int64_t* m_out) {
  CHECK_CTX(x);
  Ctx& c = x->c;
  if (!z || nslots < 1 || nslots > c.N / 2 || !m_out) return set_err(SECPE_EINVAL, "bad arguments");
  const int N = c.N;
  std::vector<double> zz(z, z + nslots);
  int64_t* m = nullptr;
  auto fn = [&](Builder& b) {
    m = (int64_t*)b.scratch(N);
    EncodeJob ej{};
    ej.z = b.put(zz);
    ej.m = m;
    ej.scale_hi = scale * 2.0 / (double)N;
    ej.scale_lo = 0.0;
    ej.nnz = nslots;
    b.encode({ej});
  };
  int rc = run_client(x, fn);
  if (rc) return rc;
  hipError_t e = hipMemcpyAsync(m_out, m, sizeof(int64_t) * N, hipMemcpyDeviceToHost, c.stream);
  if (e != hipSuccess) return hip_fail("hipMemcpyAsync", e);
  return sync(c);
}

// ---------------------------------------------------------------------------
// measurement
// ---------------------------------------------------------------------------
extern "C" int secpe_profile_begin(secpe_ctx* x, int kind) {
  CHECK_CTX(x);
  if (kind < 0 || kind >= PROF_NKINDS) return set_err(SECPE_EINVAL, "bad profile kind");
  int rc = sync(x->c);
  if (rc) return rc;
  x->c.prof_kind = kind;
  x->c.prof_used = 0;
  x->c.prof_launches = 0;
  x->c.prof_units = 0;
  x->c.prof_units_shared = 0;
  return 0;
}

extern "C" int secpe_profile_end(secpe_ctx* x, int64_t* launches, double* total_ms, int64_t* units,
                                 int64_t* units_shared) {
  CHECK_CTX(x);
  Ctx& c = x->c;
  int rc = sync(c);
  if (rc) return rc;
  double ms = 0.0;
  c.seg_ms.clear();
  if (c.prof_kind == PROF_SEGMENTS) {
    // consecutive marks: every interval between two events in order
    for (size_t i = 0; i + 1 < c.prof_used; ++i) {
      float t = 0.0f;
      if (hipEventElapsedTime(&t, c.prof_pool[i], c.prof_pool[i + 1]) != hipSuccess) t = 0.0f;
      c.seg_ms.push_back(t);
      ms += t;
    }
  } else {
    for (size_t i = 0; i + 1 < c.prof_used; i += 2) {
      float t = 0.0f;
      if (hipEventElapsedTime(&t, c.prof_pool[i], c.prof_pool[i + 1]) == hipSuccess) ms += t;
    }
  }
  if (launches) *launches = c.prof_launches;
  if (total_ms) *total_ms = ms;
  if (units) *units = c.prof_units;
  if (units_shared) *units_shared = c.prof_units_shared;
  c.prof_kind = -1;
  c.prof_used = 0;
  return 0;
}

extern "C" int secpe_profile_segments(const secpe_ctx* x, double* ms, int cap) {
  CHECK_CTX(x);
  const std::vector<double>& v = x->c.seg_ms;
  for (int i = 0; i < cap && i < (int)v.size(); ++i) ms[i] = v[i];
  return (int)v.size();
}

static void set_candidate(Ctx& c, int i) {
  c.modup_eg = (i & 1) ? 2 : 4;
  c.ntt_chunk_bytes = (i & 2) ? ((size_t)128 << 20) : 0;
  c.ntt_tiles = (i >> 2) & 7;
  c.moddown_eg = (i & 32) ? 2 : 4;
}

extern "C" int secpe_set_schedule(secpe_ctx* x, int candidate) {
  CHECK_CTX(x);
  if (candidate < 0 || candidate >= SECPE_AUTOTUNE_CANDIDATES) return set_err(SECPE_EINVAL, "no such schedule");
  drop_graphs(x->c);
  set_candidate(x->c, candidate);
  return 0;
}

extern "C" int secpe_autotune(secpe_ctx* x, const secpe_key_owner* owner, int n, const secpe_ct* in, const int* K,
                              const int* C, const double* dmin, const double* dmax, const uint64_t* rs, void* ws,
                              size_t ws_bytes, secpe_ct* out, int* chosen, double* ms, int cap) {
  CHECK_CTX(x);
  if (!chosen) return set_err(SECPE_EINVAL, "null argument");
  Ctx& c = x->c;
  // captured graphs bake in the schedule they were recorded with
  drop_graphs(c);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    if (e0) (void)hipEventDestroy(e0);
    return set_err(SECPE_EDEVICE, "hipEventCreate failed");
  }
  for (int i = 0; ms && i < cap; ++i) ms[i] = 0.0;
  int rc = 0;
  // the faster of two evaluations of the batch under candidate i
  auto time_candidate = [&](int i, float* out_ms) {
    set_candidate(c, i);
    float best = 0.0f;
    for (int rep = 0; rep < 2 && !rc; ++rep) {
      float t = 0.0f;
      (void)hipEventRecord(e0, c.stream);
      rc = secpe_eval_argmax_batch(x, owner, n, in, K, C, dmin, dmax, rs, ws, ws_bytes, out, 0);
      (void)hipEventRecord(e1, c.stream);
      if (!rc && hipEventSynchronize(e1) == hipSuccess) (void)hipEventElapsedTime(&t, e0, e1);
      if (rep == 0 || t < best) best = t;
    }
    *out_ms = best;
    if (!rc && ms && i < cap) ms[i] = best;
  };
  // coordinate search: from the default schedule, each knob (one bit of the
  // candidate index) is flipped in turn and kept when the batch gets faster
  int best = 0;
  float best_ms = 0.0f;
  time_candidate(0, &best_ms);
  for (int bit = 0; bit < SECPE_AUTOTUNE_KNOBS && !rc; ++bit) {
    const int cand = best ^ (1 << bit);
    float t = 0.0f;
    time_candidate(cand, &t);
    if (!rc && t < best_ms) {
      best = cand;
      best_ms = t;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc) return rc;
  set_candidate(c, best);
  *chosen = best;
  return 0;
}

extern "C" int secpe_ntt_cts(secpe_ctx* x, const secpe_ct* cts, int n, int inverse) {
  CHECK_CTX(x);
  Ctx& c = x->c;
  if (n < 1 || !cts) return set_err(SECPE_EINVAL, "bad arguments");
  for (int i = 0; i < n; ++i)
    if (!cts[i].data || cts[i].level < 0 || cts[i].level >= c.n_q) return set_err(SECPE_EINVAL, "bad ciphertext");
  return run_build(x, nullptr, 0, [&](Builder& b) {
    std::vector<NttJob> v;
    for (int i = 0; i < n; ++i) {
      double* d = (double*)cts[i].data;
      const int nl = cts[i].level + 1;
      v.push_back(NttJob{d, d, nl, nl, 0, 0});
      v.push_back(NttJob{d + (size_t)c.n_q * c.N, d + (size_t)c.n_q * c.N, nl, nl, 0, 0});
    }
    b.ntt(v, inverse != 0);
  });
}

extern "C" size_t secpe_rotate_workspace_bytes(secpe_ctx* x, int n) {
  if (!x || n < 1) return 0;
  Ctx& c = x->c;
  std::vector<CT> in(n);
  std::vector<int64_t> st(n, 1);
  for (int i = 0; i < n; ++i) {
    in[i].d = (double*)(uintptr_t)0x200000000000ull;
    in[i].level = c.n_q - 1;
    in[i].scale = 1.0;
  }
  Builder dry(c, (char*)(uintptr_t)0x100000000000ull, (size_t)1 << 44, (char*)(uintptr_t)0x400000000000ull,
              (size_t)1 << 40, true);
  dry.rotate(in, st);
  return dry.need_bytes() + 4096;
}

extern "C" int secpe_rotate_batch(secpe_ctx* x, int n, const secpe_ct* in, const int64_t* steps, void* ws,
                                  size_t ws_bytes, secpe_ct* out) {
  CHECK_CTX(x);
  Ctx& c = x->c;
  if (n < 1 || !in || !steps || !out || !ws) return set_err(SECPE_EINVAL, "bad arguments");
  for (int i = 0; i < n; ++i)
    if (!in[i].data || !out[i].data || in[i].level < 0 || in[i].level >= c.n_q)
      return set_err(SECPE_EINVAL, "bad ciphertext");
  std::vector<CT> res;
  int rc = run_build(x, (char*)ws, ws_bytes, [&](Builder& b) {
    std::vector<CT> v;
    std::vector<int64_t> st(steps, steps + n);
    for (int i = 0; i < n; ++i) v.push_back(to_ct(&in[i]));
    res = b.rotate(v, st);
    if (b.err_code) return;
    std::vector<EwJob> cp;
    for (int i = 0; i < n; ++i) {
      EwJob e{};
      e.o0 = (double*)out[i].data;
      e.o1 = (double*)out[i].data + (size_t)c.n_q * c.N;
      e.a0 = b.c0(res[i]);
      e.a1 = b.c1(res[i]);
      e.n_limbs = res[i].level + 1;
      e.n_chain = res[i].level + 1;
      e.op = EW_COPY;
      cp.push_back(e);
    }
    b.ew(cp);
  });
  if (rc) return rc;
  for (int i = 0; i < n; ++i) { out[i].level = res[i].level; out[i].scale = res[i].scale; }
  return 0;
}

// ---------------------------------------------------------------------------
// serving
// ---------------------------------------------------------------------------
struct secpe_server {
  secpe_ctx* x = nullptr;
  const double* refresh_sk = nullptr;   // the key owner's secret, or null
  char* ws = nullptr;
  size_t ws_bytes = 0;
  int max_active = 0;
  SlotPool pool;
  ArgmaxProgram prog;
  struct Req {
    ArgmaxQuery q;
    int slots = 0;
  };
  std::deque<std::unique_ptr<Req>> pending;
  std::map<ArgmaxQuery*, std::unique_ptr<Req>> active;
  std::map<std::pair<int, int>, std::pair<int, size_t>> need;  // (K, C) -> (peak slots, per-item scratch)
  std::map<std::pair<int, int>, int64_t> refreshes;            // (K, C) -> refreshes of one request
  int reserved_slots = 0;
  size_t item_scratch = 0;
  char* arena = nullptr;
  size_t arena_bytes = 0;
  uint64_t next_ticket = 1;
  bool broken = false;
  bool launched = false;                // a submission awaits secpe_server_collect
  std::vector<ArgmaxQuery*> finishing;  // requests that complete in it
  struct Done {
    uint64_t ticket;
    int level;
    double scale;
  };
  std::deque<Done> unreported;          // completed beyond a caller's 'cap', reported next
};

static std::pair<int, size_t> request_need(secpe_ctx* x, int K, int C, int64_t* refreshes = nullptr) {
  Ctx& c = x->c;
  std::vector<ArgmaxQuery> q(1);
  q[0].in.d = (double*)(uintptr_t)0x200000000000ull;
  q[0].in.level = c.n_q - 1;
  q[0].in.scale = ldexp(1.0, c.log_scale);
  q[0].out.d = (double*)(uintptr_t)0x300000000000ull;
  q[0].K = K;
  q[0].C = C;
  q[0].d_min = -1.0;
  q[0].d_max = 1.0;
  q[0].refresh_seed = 0;
  Builder dry(c, (char*)(uintptr_t)0x100000000000ull, (size_t)1 << 44, (char*)(uintptr_t)0x400000000000ull,
              (size_t)1 << 40, true);
  build_argmax(dry, q);
  if (dry.err_code) return {-1, 0};
  if (refreshes) *refreshes = dry.counters[4];
  return {dry.peak_slots(), dry.peak_scratch()};
}

extern "C" size_t secpe_server_request_bytes(secpe_ctx* x, int K, int C) {
  if (!x || K < 1 || C < 1) return 0;
  auto n = request_need(x, K, C);
  if (n.first < 0) return 0;
  return (size_t)n.first * x->c.ct_bytes() + n.second;
}

extern "C" int secpe_server_create(secpe_ctx* x, const secpe_key_owner* owner, void* ws_dev, size_t ws_bytes,
                                   int max_active, secpe_server** out) {
  CHECK_CTX(x);
  if (!ws_dev || !out || max_active < 1) return set_err(SECPE_EINVAL, "bad server arguments");
  const double* rsk = nullptr;
  int rc = owner_sk(x, owner, &rsk);
  if (rc) return rc;
  secpe_server* s = new secpe_server();
  s->x = x;
  s->refresh_sk = rsk;
  s->ws = (char*)ws_dev;
  s->ws_bytes = ws_bytes & ~size_t(255);
  s->max_active = max_active;
  s->arena_bytes = (size_t)64 << 20;
  hipError_t e = hipMalloc((void**)&s->arena, s->arena_bytes);
  if (e != hipSuccess) { delete s; return hip_fail("hipMalloc", e); }
  *out = s;
  return 0;
}

extern "C" void secpe_server_destroy(secpe_server* s) {
  if (!s) return;
  (void)sync(s->x->c);
  if (s->arena) (void)hipFree(s->arena);
  delete s;
}

extern "C" int secpe_server_submit(secpe_server* s, const secpe_ct* in, int K, int C, double d_min, double d_max,
                                   uint64_t refresh_seed, void* out_data, uint64_t* ticket) {
  if (!s) return set_err(SECPE_EINVAL, "null server");
  if (s->broken) return set_err(SECPE_EDEVICE, "server stopped after an error");
  if (!out_data) return set_err(SECPE_EINVAL, "null output buffer");
  int rc = check_queries(s->x, 1, in, &K, &C, &d_min, &d_max);
  if (rc) return rc;
  auto key = std::make_pair(ilog2_ceil(K), ilog2_ceil(C));
  auto it = s->need.find(key);
  if (it == s->need.end()) {
    int64_t nr = 0;
    auto n = request_need(s->x, K, C, &nr);
    if (n.first < 0) return set_err(SECPE_EINVAL, "request cannot be planned");
    it = s->need.emplace(key, n).first;
    s->refreshes[key] = nr;
  }
  // a request that must refresh is refused up front without a key owner
  if (s->refreshes[key] > 0 && !s->refresh_sk && !s->x->c.boot_mode)
    return set_err(SECPE_ENOLEVEL, "request needs a refresh and the server has no key owner");
  const size_t alone = (size_t)it->second.first * s->x->c.ct_bytes() + it->second.second;
  if (alone > s->ws_bytes) return set_err(SECPE_ENOMEM, "request does not fit the server workspace");
  std::unique_ptr<secpe_server::Req> r(new secpe_server::Req());
  r->q.in = to_ct(in);
  r->q.K = K;
  r->q.C = C;
  r->q.d_min = d_min;
  r->q.d_max = d_max;
  r->q.refresh_seed = refresh_seed;
  r->q.out.d = (double*)out_data;
  r->q.ticket = s->next_ticket++;
  r->slots = it->second.first;
  if (ticket) *ticket = r->q.ticket;
  s->pending.push_back(std::move(r));
  return 0;
}

extern "C" int secpe_server_launch(secpe_server* s) {
  if (!s) return set_err(SECPE_EINVAL, "null server");
  if (s->broken) return set_err(SECPE_EDEVICE, "server stopped after an error");
  if (s->launched) return set_err(SECPE_EINVAL, "collect the previous launch first");
  Ctx& c = s->x->c;
  // admission: the admitted set's slots plus one round's scratch must fit
  while (!s->pending.empty() && (int)s->active.size() < s->max_active) {
    secpe_server::Req* r = s->pending.front().get();
    auto n = s->need[std::make_pair(ilog2_ceil(r->q.K), ilog2_ceil(r->q.C))];
    const size_t item = s->active.empty() ? n.second : std::max(s->item_scratch, n.second);
    const size_t want = (size_t)(s->reserved_slots + r->slots) * c.ct_bytes() + (s->active.size() + 1) * item;
    if (want > s->ws_bytes) break;
    Builder probe(c, s->ws, s->ws_bytes, s->arena, s->arena_bytes, true, &s->pool);
    probe.refresh_sk = s->refresh_sk;
    if (!s->prog.add(probe, &r->q)) return set_err(SECPE_EINVAL, probe.err);
    s->item_scratch = item;
    s->reserved_slots += r->slots;
    s->active[&r->q] = std::move(s->pending.front());
    s->pending.pop_front();
  }
  if (s->active.empty()) return 0;
  Builder b(c, s->ws, s->ws_bytes, s->arena, s->arena_bytes, false, &s->pool);
  b.refresh_sk = s->refresh_sk;
  std::vector<ArgmaxQuery*> done = s->prog.round(b, true);
  // At light load a round is a few small launches, shorter than the host
  // round trip that follows it: further rounds join the same submission
  // until a request completes or the batch holds about 96 key-switches
  // (a few ms of GPU time, the longest a new arrival then waits for
  // admission).  Each request still advances through its own steps in
  // order, so results are unchanged.
  for (int r = 1; r < 64 && done.empty() && !b.err_code && s->prog.active() && b.counters[3] < 96 &&
                  b.counters[7] < 1024 && b.blob_bytes() < s->arena_bytes / 4;
       ++r)
    done = s->prog.round(b, true);
  if (b.err_code) { s->broken = true; return set_err(b.err_code, b.err); }
  if (b.arena_overflow()) { s->broken = true; return set_err(SECPE_ENOMEM, "server descriptor arena overflow"); }
  int rc = submit(c, b, s->arena, s->arena_bytes);
  if (rc) { s->broken = true; return set_err(SECPE_EDEVICE, "kernel submission failed"); }
  memcpy(c.counters, b.counters, sizeof(c.counters));
  c.ks_alg_limbs = b.ks_alg_limbs;
  s->finishing = std::move(done);
  s->launched = true;
  return 0;
}

extern "C" int secpe_server_collect(secpe_server* s, int cap, int* n_done, uint64_t* tickets, int* levels,
                                    double* scales, int* n_active, int* n_pending) {
  if (!s) return set_err(SECPE_EINVAL, "null server");
  if (n_done) *n_done = 0;
  if (s->launched) {
    s->launched = false;
    int rc = sync(s->x->c);
    if (rc) { s->broken = true; return rc; }
    for (ArgmaxQuery* q : s->finishing) {
      s->unreported.push_back({q->ticket, q->out.level, q->out.scale});
      auto it = s->active.find(q);
      if (it != s->active.end()) {
        s->reserved_slots -= it->second->slots;
        s->active.erase(it);
      }
    }
    s->finishing.clear();
    // the per-request scratch reservation follows the requests still active
    s->item_scratch = 0;
    for (auto& a : s->active)
      s->item_scratch = std::max(
          s->item_scratch, s->need[std::make_pair(ilog2_ceil(a.second->q.K), ilog2_ceil(a.second->q.C))].second);
  }
  int k = 0;
  for (; k < cap && !s->unreported.empty(); ++k) {
    const secpe_server::Done& d = s->unreported.front();
    if (tickets) tickets[k] = d.ticket;
    if (levels) levels[k] = d.level;
    if (scales) scales[k] = d.scale;
    s->unreported.pop_front();
  }
  if (n_done) *n_done = k;
  if (n_active) *n_active = (int)s->active.size();
  if (n_pending) *n_pending = (int)s->pending.size();
  return 0;
}

extern "C" int secpe_server_ready(secpe_server* s) {
  if (!s) return set_err(SECPE_EINVAL, "null server");
  if (!s->launched) return 1;
  Ctx& c = s->x->c;
  hipError_t e = hipStreamQuery(c.stream);
  if (e == hipSuccess) return 1;
  if (e == hipErrorNotReady) return 0;
  s->broken = true;
  return hip_fail("stream query", e);
}

extern "C" int secpe_server_step(secpe_server* s, int cap, int* n_done, uint64_t* tickets, int* levels, double* scales,
                                 int* n_active, int* n_pending) {
  if (n_done) *n_done = 0;
  int rc = secpe_server_launch(s);
  if (rc) return rc;
  return secpe_server_collect(s, cap, n_done, tickets, levels, scales, n_active, n_pending);
}

// ---------------------------------------------------------------------------
// bootstrapping
// ---------------------------------------------------------------------------
static int64_t floor_div64(int64_t a, int64_t b) { return a >= 0 ? a / b : -((-a + b - 1) / b); }

// levels, input scales and plaintext scales of every group (no slot vectors);
// the sparse-slot transforms (log_ns = log2 n) have the same levels and scales
static void boot_plan_groups(Ctx& c, int log_ns, std::vector<BootGroup>& cts, std::vector<BootGroup>& stc) {
  const double delta = ldexp(1.0, c.log_scale);
  const int top = c.n_q - 1;
  int k = 0;
  while ((1 << k) < c.boot_deg + 1) ++k;
  cts.clear();
  stc.clear();
  for (int inv = 1; inv >= 0; --inv) {
    int lvl0 = top;
    double s0 = (double)c.mod[0];
    if (!inv) {
      // EvalMod: the Chebyshev sum lands on Delta one level below T_deg, then
      // each double angle takes s to s^2 / q_l
      lvl0 = top - c.boot_groups - k - 1;
      s0 = delta;
      for (int i = 0; i < c.boot_r; ++i) {
        s0 = s0 * s0 / (double)c.mod[lvl0];
        --lvl0;
      }
    }
    std::vector<BootGroup>& out = inv ? cts : stc;
    for (int g = 0; g < c.boot_groups; ++g) {
      BootGroupTable t = boot_group_geometry(c.log_n, log_ns, c.boot_groups, inv, g);
      BootGroup G;
      G.inverse = inv;
      G.g = g;
      G.log_ns = log_ns;
      G.level = lvl0 - g;
      G.delta = t.delta;
      G.n1 = t.n1;
      G.E = t.E;
      // CoeffToSlot keeps 2^5 Delta until its last group: its first groups
      // carry the large ModRaise overflow, so their plaintexts get the larger scale
      G.out_scale = (inv && g < c.boot_groups - 1) ? ldexp(1.0, c.log_scale + 5) : delta;
      G.in_scale = g == 0 ? s0 : out.back().out_scale;
      double ps = G.out_scale * (double)c.mod[G.level];
      ps = ps / G.in_scale;
      G.pscale = ps;
      out.push_back(G);
    }
  }
}
static int ilog2(int v) {
  int k = 0;
  while ((1 << k) < v) ++k;
  return k;
}
static void boot_plan(Ctx& c) {
  boot_plan_groups(c, c.log_n - 1, c.boot_cts, c.boot_stc);
  c.boot_cts_sp.clear();
  c.boot_stc_sp.clear();
  if (c.boot_sparse > 0) boot_plan_groups(c, ilog2(c.boot_sparse), c.boot_cts_sp, c.boot_stc_sp);
}

extern "C" int secpe_set_boot(secpe_ctx* x, const secpe_boot_params* bp, int* out_level) {
  CHECK_CTX(x);
  if (!bp) return set_err(SECPE_EINVAL, "null parameters");
  Ctx& c = x->c;
  if (bp->secret_h < 0 || bp->secret_h > c.N) return set_err(SECPE_EINVAL, "secret_h must be in [0, N]");
  drop_graphs(c);
  c.secret_h = bp->secret_h;
  c.boot_cts.clear();
  c.boot_stc.clear();
  c.boot_cts_sp.clear();
  c.boot_stc_sp.clear();
  c.boot_sparse = 0;
  c.boot_pack_min = 0;
  c.keys_perm.clear();
  c.boot_ready = false;
  c.boot_mono = nullptr;
  c.boot_mode = 0;
  c.boot_out_level = -1;
  c.refresh_level = c.refresh_level_set;
  if (out_level) *out_level = -1;
  if (bp->K <= 0) return 0;
  if (bp->deg < 1 || ((bp->deg + 1) & bp->deg) || bp->r < 0 || bp->groups < 1 || bp->groups > c.log_n - 1 ||
      bp->ratio < 1 || bp->ratio > 40)
    return set_err(SECPE_EINVAL, "bad bootstrapping parameters");
  // the sparse-slot bootstrap: a power of two with 2n <= N/2 and a stage per group
  const int sp = bp->sparse_slots;
  if (sp != 0 && (sp < 0 || (sp & (sp - 1)) || 2 * sp > c.N / 2 || ilog2(sp) < bp->groups))
    return set_err(SECPE_EINVAL, "sparse_slots must be 0 or a power of two n with 2n <= N/2 and log2 n >= groups");
  if (bp->pack_min != 0 && (bp->pack_min < 2 || sp == 0))
    return set_err(SECPE_EINVAL, "pack_min must be 0, or at least 2 with sparse_slots set");
  int k = 0;
  while ((1 << k) < bp->deg + 1) ++k;
  const int out = c.n_q - 1 - (2 * bp->groups + k + 1 + bp->r);
  if (out < c.min_level) return set_err(SECPE_EINVAL, "modulus chain too short for bootstrapping");
  c.boot_K = bp->K;
  c.boot_r = bp->r;
  c.boot_deg = bp->deg;
  c.boot_ratio = bp->ratio;
  c.boot_groups = bp->groups;
  c.boot_cheb.assign(bp->deg + 1, 0.0);
  boot_cheb_coeffs(bp->K, bp->r, bp->deg, c.boot_cheb.data());
  c.boot_out_level = out;
  c.boot_mode = bp->refresh ? 1 : 0;
  c.boot_sparse = sp;
  c.boot_pack_min = bp->pack_min;
  if (c.boot_mode) c.refresh_level = out;
  boot_plan(c);
  if (out_level) *out_level = out;
  return 0;
}

extern "C" int secpe_boot_steps(const secpe_ctx* x, int64_t* out, int cap) {
  CHECK_CTX(x);
  const Ctx& c = x->c;
  if (c.boot_out_level < 0) return set_err(SECPE_EINVAL, "bootstrapping is not configured");
  const int64_t S = c.N / 2;
  std::vector<int64_t> st;
  for (int inv = 0; inv < 2; ++inv)
    for (int g = 0; g < c.boot_groups; ++g) {
      BootGroupTable t = boot_group_geometry(c.log_n, c.log_n - 1, c.boot_groups, inv, g);
      for (int b = 1; b < t.n1; ++b) st.push_back((int64_t)t.delta * b % S);
      // offsets are delta e with |e| <= 2^len - 1, centred in [-E/2, E/2)
      const int64_t span = ((int64_t)1 << t.len) - 1;
      const int64_t elo = std::max(-span, -(int64_t)t.E / 2), ehi = std::min(span, (int64_t)t.E / 2 - 1);
      for (int64_t G = floor_div64(elo, t.n1); G <= floor_div64(ehi, t.n1); ++G)
        if (G) st.push_back((((int64_t)t.delta * t.n1 * G) % S + S) % S);
    }
  if (c.boot_sparse > 0) {
    // the sparse transforms: baby steps, and the giant steps of the offsets
    // their (small) tables hold; the traces; RotR(n)
    for (int inv = 0; inv < 2; ++inv)
      for (int g = 0; g < c.boot_groups; ++g) {
        BootGroupTable t = boot_group_table(c.log_n, ilog2(c.boot_sparse), c.boot_groups, c.boot_K, c.boot_ratio, inv, g);
        for (int b = 1; b < t.n1; ++b) st.push_back((int64_t)t.delta * b % S);
        for (const BootDiag& d : t.diags) {
          int64_t e = d.off / t.delta;
          if (e >= t.E / 2) e -= t.E;
          const int64_t G = floor_div64(e, t.n1);
          if (G) st.push_back((((int64_t)t.delta * t.n1 * G) % S + S) % S);
        }
      }
    for (int64_t r = c.boot_sparse; r < S; r *= 2) st.push_back(r);
    st.push_back(S - c.boot_sparse);
  }
  std::sort(st.begin(), st.end());
  st.erase(std::unique(st.begin(), st.end()), st.end());
  st.erase(std::remove_if(st.begin(), st.end(), [&](int64_t v) { return v % S == 0; }), st.end());
  st.push_back(kConjStep);
  for (size_t i = 0; i < st.size() && (int)i < cap; ++i) out[i] = st[i];
  return (int)st.size();
}

// offsets present in a group: every delta e, e centred in [-E/2, E/2) with
// |e| <= 2^len - 1 (sums of the stages' 0, +-m/2), as slot offsets mod S
static std::vector<int64_t> boot_group_es(const BootGroup& G, int len) {
  const int64_t span = ((int64_t)1 << len) - 1;
  const int64_t elo = std::max(-span, -(int64_t)G.E / 2), ehi = std::min(span, (int64_t)G.E / 2 - 1);
  std::vector<int64_t> es;
  for (int64_t e = elo; e <= ehi; ++e) es.push_back(e);
  return es;
}

// Galois elements of the sparse-slot transforms' baby steps that have a key
static std::vector<uint64_t> sparse_baby_galois(const Ctx& c) {
  std::vector<uint64_t> gs;
  const int64_t S = c.N / 2;
  for (const std::vector<BootGroup>* list : {&c.boot_cts_sp, &c.boot_stc_sp})
    for (const BootGroup& G : *list)
      for (int b = 1; b < G.n1; ++b) {
        const uint64_t g = c.galois((int64_t)G.delta * b % S);
        if (c.keys.count(g)) gs.push_back(g);
      }
  std::sort(gs.begin(), gs.end());
  gs.erase(std::unique(gs.begin(), gs.end()), gs.end());
  return gs;
}

// g^-1 mod 2N for odd g (Newton's iteration doubles the correct low bits)
static uint64_t galois_inverse(uint64_t g, uint64_t m2n) {
  uint64_t v = g;
  for (int i = 0; i < 6; ++i) v *= 2 - g * v;
  return v & (m2n - 1);
}

extern "C" size_t secpe_boot_key_bytes(secpe_ctx* x) {
  if (!x || x->c.boot_out_level < 0) return 0;
  Ctx& c = x->c;
  size_t total = 2 * (size_t)c.n_q * c.limb_bytes();
  for (int inv = 0; inv < 2; ++inv)
    for (const BootGroup& G : inv ? c.boot_cts : c.boot_stc) {
      const int len = boot_group_geometry(c.log_n, c.log_n - 1, c.boot_groups, inv, G.g).len;
      total += boot_group_es(G, len).size() * (size_t)(G.level + 1) * c.limb_bytes();
    }
  for (int inv = 0; inv < 2; ++inv)
    for (const BootGroup& G : inv ? c.boot_cts_sp : c.boot_stc_sp) {
      const size_t nd =
          boot_group_table(c.log_n, G.log_ns, c.boot_groups, c.boot_K, c.boot_ratio, inv, G.g).diags.size();
      total += nd * (size_t)(G.level + 1) * c.limb_bytes();
    }
  // the permuted keys of the sparse transforms' baby steps
  total += sparse_baby_galois(c).size() * c.key_bytes();
  return total;
}

extern "C" int secpe_boot_setup(secpe_ctx* x, void* buf_dev, size_t bytes) {
  CHECK_CTX(x);
  Ctx& c = x->c;
  if (c.boot_out_level < 0) return set_err(SECPE_EINVAL, "bootstrapping is not configured");
  if (!buf_dev || bytes < secpe_boot_key_bytes(x)) return set_err(SECPE_EINVAL, "boot key buffer too small");
  const int N = c.N, S = N / 2;
  double* cur = (double*)buf_dev;
  c.boot_ready = false;
  // X^(N/2) and -X^(N/2) in the NTT domain, every chain limb
  {
    double* mono = cur;
    cur += 2 * (size_t)c.n_q * N;
    std::vector<int64_t> mp(N, 0), mn(N, 0);
    mp[N / 2] = 1;
    mn[N / 2] = -1;
    auto fn = [&](Builder& b) {
      const int64_t* sp = (const int64_t*)b.put_bytes(mp.data(), sizeof(int64_t) * N);
      const int64_t* sn = (const int64_t*)b.put_bytes(mn.data(), sizeof(int64_t) * N);
      double* d1 = mono + (size_t)c.n_q * N;
      b.intspread({IntSpreadJob{sp, mono, c.n_q, c.n_q}, IntSpreadJob{sn, d1, c.n_q, c.n_q}});
      b.ntt({NttJob{mono, mono, c.n_q, c.n_q, 0, 0}, NttJob{d1, d1, c.n_q, c.n_q, 0, 0}}, false);
    };
    int rc = run_client(x, fn);
    if (rc) return rc;
    c.boot_mono = mono;
  }
  for (int which = 0; which < 4; ++which) {
    const int inv = which & 1 ? 0 : 1;
    std::vector<BootGroup>& list = which < 2 ? (inv ? c.boot_cts : c.boot_stc) : (inv ? c.boot_cts_sp : c.boot_stc_sp);
    for (BootGroup& G : list) {
      BootGroupTable t = boot_group_table(c.log_n, G.log_ns, c.boot_groups, c.boot_K, c.boot_ratio, inv, G.g);
      const int ns = t.ns;
      G.e.clear();
      G.pt.clear();
      // the nonzero entries of each pre-rotated diagonal as (5^slot mod 2N, re, im)
      std::vector<std::vector<double>> re, im;
      std::vector<std::vector<uint32_t>> gs;
      std::vector<uint32_t> g5(S);
      for (int p = 0, v = 1; p < S; ++p, v = (int)((uint64_t)v * 5 % (2ull * N))) g5[p] = (uint32_t)v;
      for (const BootDiag& d : t.diags) {
        int64_t e = d.off / G.delta;
        if (e >= G.E / 2) e -= G.E;
        const int64_t gg = floor_div64(e, G.n1);
        // the diagonal, pre-rotated by delta n1 gg, repeats with period ns
        const int64_t shift = (((int64_t)G.delta * G.n1 * gg) % ns + ns) % ns;
        std::vector<double> r, i2;
        std::vector<uint32_t> gv;
        for (int p = 0; p < S; ++p) {
          const int src = (int)(((int64_t)(p % ns) - shift + ns) % ns);
          if (d.re[src] == 0.0 && d.im[src] == 0.0) continue;
          r.push_back(d.re[src]);
          i2.push_back(d.im[src]);
          gv.push_back(g5[p]);
        }
        if (r.empty()) {  // an all-zero diagonal still takes part (as zero)
          r.push_back(0.0);
          i2.push_back(0.0);
          gv.push_back(1u);
        }
        G.e.push_back(e);
        G.pt.push_back(cur);
        cur += (size_t)(G.level + 1) * N;
        if ((char*)cur > (char*)buf_dev + bytes) return set_err(SECPE_EINVAL, "boot key buffer too small");
        re.push_back(std::move(r));
        im.push_back(std::move(i2));
        gs.push_back(std::move(gv));
      }
      const int nl = G.level + 1;
      auto fn = [&](Builder& b) {
        std::vector<EncodeJob> j_enc;
        std::vector<FftEncJob> j_fft;
        std::vector<IntSpreadJob> j_sp;
        std::vector<NttJob> j_ntt;
        // diagonals with many nonzero slots go through one length-2N FFT each
        // (O(N log N) instead of O(N nnz)), in groups that share one buffer
        constexpr int kFftMinSlots = 256, kFftGroup = 32;
        double* fft_buf = nullptr;
        for (size_t i = 0; i < G.pt.size(); ++i) {
          int64_t* m = (int64_t*)b.scratch(N);
          const int nnz = (int)re[i].size();
          const double sc = G.pscale * 2.0 / (double)N;   // exact: N is a power of two
          if (nnz > kFftMinSlots) {
            if (!fft_buf) fft_buf = b.scratch((size_t)kFftGroup * 16 * N);
            FftEncJob fj{};
            fj.z = b.put(re[i]);
            fj.zi = b.put(im[i]);
            fj.gs = b.put(gs[i]);
            fj.nnz = nnz;
            fj.m = m;
            fj.buf = fft_buf + (size_t)(j_fft.size() % kFftGroup) * 16 * N;
            fj.scale_hi = sc;
            fj.scale_lo = 0.0;
            j_fft.push_back(fj);
          } else {
            EncodeJob ej{};
            ej.z = b.put(re[i]);
            ej.zi = b.put(im[i]);
            ej.gs = b.put(gs[i]);
            ej.nnz = nnz;
            ej.m = m;
            ej.scale_hi = sc;
            ej.scale_lo = 0.0;
            j_enc.push_back(ej);
          }
          double* pt = (double*)G.pt[i];
          j_sp.push_back(IntSpreadJob{m, pt, nl, nl});
          j_ntt.push_back(NttJob{pt, pt, nl, nl, 0, 0});
        }
        b.encode(j_enc);
        // groups run one after another on the stream, so they can share the buffer
        for (size_t g0 = 0; g0 < j_fft.size(); g0 += kFftGroup) {
          const size_t g1 = std::min(j_fft.size(), g0 + (size_t)kFftGroup);
          b.fft_encode(std::vector<FftEncJob>(j_fft.begin() + g0, j_fft.begin() + g1));
        }
        b.intspread(j_sp);
        b.ntt(j_ntt, false);
      };
      int rc = run_client(x, fn);
      if (rc) return rc;
      rc = sync(c);
      if (rc) return rc;
    }
  }
  // each sparse baby step's key with every limb taken through X -> X^(g^-1);
  // destinations are laid out here, once (run_client builds fn twice: a dry
  // run to size the workspace, then the real one)
  c.keys_perm.clear();
  {
    const std::vector<uint64_t> gs = sparse_baby_galois(c);
    const int nl = c.dnum * 2 * c.n_mod;
    std::vector<std::pair<uint64_t, double*>> made;
    for (uint64_t g : gs) {
      made.push_back({g, cur});
      cur += (size_t)nl * N;
    }
    if ((char*)cur > (char*)buf_dev + bytes) return set_err(SECPE_EINVAL, "boot key buffer too small");
    auto fn = [&](Builder& b) {
      std::vector<AutoJob> j;
      for (auto& kv : made)
        j.push_back(AutoJob{c.keys.at(kv.first), kv.second, nl, nl,
                            (uint32_t)galois_inverse(kv.first, 2ull * (uint64_t)N), 0});
      b.automorph(j);
    };
    if (!gs.empty()) {
      int rc = run_client(x, fn);
      if (rc) return rc;
      rc = sync(c);
      if (rc) return rc;
      for (auto& kv : made) c.keys_perm[kv.first] = kv.second;
    }
  }
  drop_graphs(c);
  c.boot_ready = true;
  return sync(c);
}

static std::vector<CT> boot_inputs(int n, const secpe_ct* in) {
  std::vector<CT> v;
  for (int i = 0; i < n; ++i) v.push_back(to_ct(&in[i]));
  return v;
}

extern "C" size_t secpe_bootstrap_workspace_bytes(secpe_ctx* x, int n) {
  if (!x || n < 1) return 0;
  if (!x->c.boot_ready) {
    set_err(SECPE_EINVAL, "bootstrapping is not set up (secpe_boot_setup)");
    return 0;
  }
  Ctx& c = x->c;
  std::vector<secpe_ct> in(n, secpe_ct{(void*)(uintptr_t)0x200000000000ull, 1, ldexp(1.0, c.log_scale)});
  size_t need = 0;
  // the largest of the full, the sparse-slot and the packed pipelines
  for (int mode = 0; mode < (c.boot_sparse > 0 ? 3 : 1); ++mode) {
    Builder dry(c, (char*)(uintptr_t)0x100000000000ull, (size_t)1 << 44, (char*)(uintptr_t)0x400000000000ull,
                (size_t)1 << 40, true);
    std::vector<CT> v = boot_inputs(n, in.data());
    // the dry build takes the set-up scales for granted
    if (mode == 2) dry.bootstrap_packed(v);
    else dry.bootstrap(v, mode == 1);
    if (dry.err_code) {
      set_err(dry.err_code, dry.err);
      return 0;
    }
    need = std::max(need, dry.need_bytes());
  }
  return need + 4096;
}

// mode 0: full-slot, 1: sparse-slot, 2: window-packed
static int bootstrap_into(secpe_ctx* x, int n, const secpe_ct* in, void* ws, size_t ws_bytes, secpe_ct* out,
                          int mode) {
  CHECK_CTX(x);
  Ctx& c = x->c;
  if (n < 1 || !in || !out || !ws) return set_err(SECPE_EINVAL, "bad bootstrap arguments");
  if (!c.boot_ready) return set_err(SECPE_EINVAL, "bootstrapping is not set up (secpe_boot_setup)");
  if (mode && c.boot_sparse <= 0) return set_err(SECPE_EINVAL, "sparse_slots is 0: no sparse-slot bootstrap");
  for (int i = 0; i < n; ++i) {
    if (!in[i].data || !out[i].data) return set_err(SECPE_EINVAL, "null ciphertext");
    if (in[i].level < 1 || in[i].level >= c.n_q) return set_err(SECPE_EINVAL, "bootstrap input needs level in [1, n_q)");
  }
  std::vector<CT> res;
  int rc = run_build(x, (char*)ws, ws_bytes, [&](Builder& b) {
    std::vector<CT> r = mode == 2 ? b.bootstrap_packed(boot_inputs(n, in)) : b.bootstrap(boot_inputs(n, in), mode == 1);
    if (b.err_code) return;
    std::vector<EwJob> j;
    for (int i = 0; i < n; ++i) {
      EwJob e{};
      e.o0 = (double*)out[i].data;
      e.o1 = (double*)out[i].data + (size_t)c.n_q * c.N;
      e.a0 = b.c0(r[i]);
      e.a1 = b.c1(r[i]);
      e.n_limbs = r[i].level + 1;
      e.n_chain = r[i].level + 1;
      e.op = EW_COPY;
      j.push_back(e);
    }
    b.ew(j);
    res = r;
  });
  if (rc) return rc;
  for (int i = 0; i < n; ++i) {
    out[i].level = res[i].level;
    out[i].scale = res[i].scale;
  }
  return 0;
}

extern "C" int secpe_bootstrap(secpe_ctx* x, int n, const secpe_ct* in, void* ws, size_t ws_bytes, secpe_ct* out) {
  return bootstrap_into(x, n, in, ws, ws_bytes, out, 0);
}

extern "C" int secpe_bootstrap_sparse(secpe_ctx* x, int n, const secpe_ct* in, void* ws, size_t ws_bytes,
                                      secpe_ct* out) {
  return bootstrap_into(x, n, in, ws, ws_bytes, out, 1);
}

extern "C" int secpe_bootstrap_packed(secpe_ctx* x, int n, const secpe_ct* in, void* ws, size_t ws_bytes,
                                      secpe_ct* out) {
  return bootstrap_into(x, n, in, ws, ws_bytes, out, 2);
}

extern "C" int secpe_op_boot_step(secpe_ctx* x, int step, const secpe_ct* a, void* ws, size_t ws_bytes, secpe_ct* out) {
  CHECK_CTX(x);
  if (!a || !a->data) return set_err(SECPE_EINVAL, "null input");
  if (step < 0 || step > 7) return set_err(SECPE_EINVAL, "unknown bootstrapping step");
  // the linear transforms and the monomials need secpe_boot_setup; EvalMod the parameters
  if (step != 0 && step != 3 && !x->c.boot_ready)
    return set_err(SECPE_EINVAL, "bootstrapping is not set up (secpe_boot_setup)");
  if (step >= 6 && x->c.boot_sparse <= 0) return set_err(SECPE_EINVAL, "sparse_slots is 0: no sparse-slot bootstrap");
  if (step == 3 && x->c.boot_out_level < 0) return set_err(SECPE_EINVAL, "bootstrapping is not configured");
  return op_to_out(x, ws, ws_bytes, out, [&](Builder& b) -> std::vector<CT> {
    const std::vector<CT> v{to_ct(a)};
    switch (step) {
      case 0: return b.mod_raise(v);
      case 1: return b.boot_transform(v, true);
      case 2: return b.boot_transform(v, false);
      case 3: return b.eval_mod(v);
      case 4: return b.mul_monomial_half(v, false);
      case 5: return b.mul_monomial_half(v, true);
      case 6: return b.boot_transform(v, true, true);
      default: return b.boot_transform(v, false, true);
    }
  });
}
