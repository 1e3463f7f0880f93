// Host runtime: RNS-CKKS context, command lists and batched homomorphic
// operations (arXiv 2502.00847, Sec. 2.2).
#include "runtime.h"

#include <math.h>
#include <string.h>

#include <algorithm>
#include <tuple>

extern "C" void secpe_cos_table_dd(int log_n, double* hi, double* lo);

namespace secpe {

// ---------------------------------------------------------------------------
// primes: chain = 1 mod 2N nearest 2^q_bits, alternately below and above;
// special = the largest = 1 mod 2N below 2^p_bits not already used
// ---------------------------------------------------------------------------
static bool miller_rabin(uint64_t n) {
  if (n < 2) return false;
  const uint64_t small[] = {2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37};
  for (uint64_t p : small)
    if (n % p == 0) return n == p;
  uint64_t d = n - 1;
  int s = 0;
  while (!(d & 1)) { d >>= 1; ++s; }
  for (uint64_t a : small) {
    uint64_t x = hpow(a, d, n);
    if (x == 1 || x == n - 1) continue;
    bool comp = true;
    for (int r = 1; r < s && comp; ++r) {
      x = hmul(x, x, n);
      if (x == n - 1) comp = false;
    }
    if (comp) return false;
  }
  return true;
}

static std::vector<uint64_t> choose_primes(int log_n, int n_q, int q_bits, int n_p, int p_bits) {
  const uint64_t step = 2ull << log_n;
  std::vector<uint64_t> out;
  uint64_t below = (1ull << q_bits) + 1 - step, above = (1ull << q_bits) + 1;
  for (int k = 0; k < n_q; ++k) {
    if (k % 2 == 0) {
      while (!miller_rabin(below)) below -= step;
      out.push_back(below);
      below -= step;
    } else {
      while (!miller_rabin(above)) above += step;
      out.push_back(above);
      above += step;
    }
  }
  uint64_t c = (1ull << p_bits) + 1 - step;
  for (int k = 0; k < n_p; ++k) {
    while (!miller_rabin(c) || std::find(out.begin(), out.end(), c) != out.end()) c -= step;
    out.push_back(c);
    c -= step;
  }
  return out;
}

static uint64_t psi_root(uint64_t q, uint64_t n) {
  // psi = x^((q-1)/2N) for a quadratic non-residue x has order exactly 2N
  for (uint64_t x = 3;; ++x)
    if (hpow(x, (q - 1) / 2, q) == q - 1) return hpow(x, (q - 1) / (2 * n), q);
}

static uint32_t bitrev(uint32_t x, int bits) {
  uint32_t r = 0;
  for (int i = 0; i < bits; ++i) r |= ((x >> i) & 1u) << (bits - 1 - i);
  return r;
}

uint64_t Ctx::galois(int64_t step) const {
  if (step == kConjStep) return 2 * (uint64_t)N - 1;
  const int64_t slots = N / 2;
  const int64_t r = ((step % slots) + slots) % slots;
  return hpow(5, (uint64_t)r, 2 * (uint64_t)N);
}

int ilog2_ceil(int v) {
  int r = 0;
  while ((1 << r) < v) ++r;
  return r;
}

static const int SECPE_EDEVICE_INTERNAL = -5;
#define HIPCHK(x)                                         \
  do {                                                    \
    if ((x) != hipSuccess) return SECPE_EDEVICE_INTERNAL; \
  } while (0)

int build_context(Ctx& c, int log_n, int n_q, int q_bits, int n_p, int p_bits, int log_scale, int dg, int df,
                  int min_level, int refresh_level, int device, hipStream_t stream) {
  c.log_n = log_n;
  c.N = 1 << log_n;
  c.n_q = n_q;
  c.n_p = n_p;
  c.alpha = n_p;
  c.dnum = (n_q + n_p - 1) / n_p;
  c.n_mod = n_q + n_p;
  c.q_bits = q_bits;
  c.p_bits = p_bits;
  c.log_scale = log_scale;
  c.dg = dg;
  c.df = df;
  c.min_level = min_level;
  c.refresh_level = (refresh_level <= 0 || refresh_level > n_q - 1) ? n_q - 1 : refresh_level;
  c.refresh_level_set = c.refresh_level;
  c.device = device;
  c.stream = stream;
  c.mod = choose_primes(log_n, n_q, q_bits, n_p, p_bits);
  const int N = c.N, nm = c.n_mod;
  // ----- host tables -----
  std::vector<double> h;
  auto alloc = [&](size_t n) {
    size_t off = h.size();
    h.resize(off + ((n + 31) & ~size_t(31)), 0.0);
    return off;
  };
  size_t o_mod = alloc(nm), o_minv = alloc(nm), o_ninv = alloc(nm), o_ninvq = alloc(nm);
  size_t o_psi = alloc((size_t)nm * N), o_psiq = alloc((size_t)nm * N);
  size_t o_ipsi = alloc((size_t)nm * N), o_ipsiq = alloc((size_t)nm * N);
  size_t o_cos_hi = alloc(2 * (size_t)N), o_cos_lo = alloc(2 * (size_t)N);
  for (int t = 0; t < nm; ++t) {
    const uint64_t q = c.mod[t];
    const double qd = (double)q;
    h[o_mod + t] = qd;
    h[o_minv + t] = 1.0 / qd;
    const uint64_t ni = hinv((uint64_t)N, q);
    h[o_ninv + t] = (double)ni;
    h[o_ninvq + t] = (double)ni / qd;
    const uint64_t psi = psi_root(q, (uint64_t)N), ipsi = hinv(psi, q);
    std::vector<uint64_t> pw(N), ipw(N);
    uint64_t a = 1, b = 1;
    for (int i = 0; i < N; ++i) { pw[i] = a; ipw[i] = b; a = hmul(a, psi, q); b = hmul(b, ipsi, q); }
    for (int k = 0; k < N; ++k) {
      const uint32_t r = bitrev((uint32_t)k, log_n);
      h[o_psi + (size_t)t * N + k] = (double)pw[r];
      h[o_psiq + (size_t)t * N + k] = (double)pw[r] / qd;
      h[o_ipsi + (size_t)t * N + k] = (double)ipw[r];
      h[o_ipsiq + (size_t)t * N + k] = (double)ipw[r] / qd;
    }
  }
  secpe_cos_table_dd(log_n, &h[o_cos_hi], &h[o_cos_lo]);
  // digit tables for every (lo, size) a level can produce
  struct DOff { size_t cinv, chat; };
  std::map<std::pair<int, int>, DOff> doff;
  for (int lo = 0; lo < n_q; lo += c.alpha) {
    for (int sz = 1; sz <= c.alpha && lo + sz <= n_q; ++sz) {
      DOff d;
      d.cinv = alloc(sz);
      d.chat = alloc((size_t)nm * sz);
      for (int i = 0; i < sz; ++i) {
        const uint64_t qi = c.mod[lo + i];
        uint64_t dh = 1;
        for (int i2 = 0; i2 < sz; ++i2)
          if (i2 != i) dh = hmul(dh, c.mod[lo + i2] % qi, qi);
        h[d.cinv + i] = (double)hinv(dh, qi);
        for (int t = 0; t < nm; ++t) {
          const uint64_t qt = c.mod[t];
          uint64_t v = 1;
          for (int i2 = 0; i2 < sz; ++i2)
            if (i2 != i) v = hmul(v, c.mod[lo + i2] % qt, qt);
          h[d.chat + (size_t)t * sz + i] = (double)v;
        }
      }
      doff[{lo, sz}] = d;
    }
  }
  // ModDown / P tables
  size_t o_mdc = alloc(c.alpha), o_mdh = alloc((size_t)n_q * c.alpha), o_mdp = alloc(n_q), o_pmq = alloc(n_q);
  for (int k = 0; k < c.alpha; ++k) {
    const uint64_t pk = c.mod[n_q + k];
    uint64_t ph = 1;
    for (int k2 = 0; k2 < c.alpha; ++k2)
      if (k2 != k) ph = hmul(ph, c.mod[n_q + k2] % pk, pk);
    h[o_mdc + k] = (double)hinv(ph, pk);
  }
  for (int t = 0; t < n_q; ++t) {
    const uint64_t q = c.mod[t];
    uint64_t P = 1;
    for (int k = 0; k < c.alpha; ++k) P = hmul(P, c.mod[n_q + k] % q, q);
    h[o_mdp + t] = (double)hinv(P, q);
    h[o_pmq + t] = (double)P;
    for (int k = 0; k < c.alpha; ++k) {
      uint64_t ph = 1;
      for (int k2 = 0; k2 < c.alpha; ++k2)
        if (k2 != k) ph = hmul(ph, c.mod[n_q + k2] % q, q);
      h[o_mdh + (size_t)t * c.alpha + k] = (double)ph;
    }
  }
  // inverse NTT feeding the fused ModUp: at level l, limb t is scaled by
  // N^-1 (D_j/q_t)^-1 mod q_t, D_j the product of the primes of t's digit
  size_t o_ytab = alloc((size_t)n_q * n_q);
  for (int l = 0; l < n_q; ++l)
    for (int t = 0; t <= l; ++t) {
      const uint64_t q = c.mod[t];
      const int lo = (t / c.alpha) * c.alpha, hi = std::min(lo + c.alpha, l + 1);
      uint64_t dh = 1;
      for (int i = lo; i < hi; ++i)
        if (i != t) dh = hmul(dh, c.mod[i] % q, q);
      h[o_ytab + (size_t)l * n_q + t] = (double)hmul(hinv(dh, q), hinv((uint64_t)c.N % q, q), q);
    }
  // merged relinearise + rescale at level l: base B = {q_l} u P
  const int nb = c.alpha + 1;
  size_t o_rrc = alloc((size_t)n_q * nb), o_rrh = alloc((size_t)n_q * n_q * nb), o_rri = alloc((size_t)n_q * n_q);
  for (int l = 1; l < n_q; ++l) {
    std::vector<int> bp(1, l);
    for (int k = 0; k < c.alpha; ++k) bp.push_back(n_q + k);
    for (int i = 0; i < nb; ++i) {
      const uint64_t b = c.mod[bp[i]];
      uint64_t bh = 1;
      for (int i2 = 0; i2 < nb; ++i2)
        if (i2 != i) bh = hmul(bh, c.mod[bp[i2]] % b, b);
      h[o_rrc + (size_t)l * nb + i] = (double)hinv(bh, b);
    }
    for (int t = 0; t < l; ++t) {
      const uint64_t q = c.mod[t];
      uint64_t all = 1;
      for (int i = 0; i < nb; ++i) {
        all = hmul(all, c.mod[bp[i]] % q, q);
        uint64_t bh = 1;
        for (int i2 = 0; i2 < nb; ++i2)
          if (i2 != i) bh = hmul(bh, c.mod[bp[i2]] % q, q);
        h[o_rrh + ((size_t)l * n_q + t) * nb + i] = (double)bh;
      }
      h[o_rri + (size_t)l * n_q + t] = (double)hinv(all, q);
    }
  }
  // the inverse transform feeding a conversion from B also applies (B/b)^-1:
  // limb b is scaled by N^-1 (B/b)^-1 mod b
  size_t o_mdy = alloc(c.alpha), o_rry = alloc((size_t)n_q * (n_q + c.alpha));
  for (int k = 0; k < c.alpha; ++k) {
    const uint64_t pk = c.mod[n_q + k];
    h[o_mdy + k] = (double)hmul((uint64_t)h[o_mdc + k], hinv((uint64_t)c.N % pk, pk), pk);
  }
  for (int l = 1; l < n_q; ++l)
    for (int i = 0; i < nb; ++i) {
      const uint64_t b = c.mod[i == 0 ? l : n_q + i - 1];
      h[o_rry + (size_t)l * (n_q + c.alpha) + l + i] =
          (double)hmul((uint64_t)h[o_rrc + (size_t)l * nb + i], hinv((uint64_t)c.N % b, b), b);
    }
  // rescale: q_l^-1 mod q_i
  size_t o_rs = alloc((size_t)n_q * n_q);
  for (int l = 1; l < n_q; ++l)
    for (int i = 0; i < l; ++i) h[o_rs + (size_t)l * n_q + i] = (double)hinv(c.mod[l] % c.mod[i], c.mod[i]);
  // CRT from limbs 0, 1
  size_t o_crt = alloc(2 * (size_t)n_q);
  for (int t = 0; t < n_q; ++t) {
    const uint64_t q = c.mod[t];
    h[o_crt + 2 * t] = (double)(c.mod[0] % q);
    h[o_crt + 2 * t + 1] = (double)hmul(c.mod[0] % q, c.mod[1] % q, q);
  }
  c.q0inv_q1 = (double)hinv(c.mod[0] % c.mod[1], c.mod[1]);
  if (const char* e = getenv("SECPE_NTT_CHUNK_MB")) c.ntt_chunk_bytes = (size_t)std::max(0L, atol(e)) << 20;
  if (const char* e = getenv("SECPE_BOOT_CHUNK")) c.boot_chunk = (int)std::max(1L, std::min(256L, atol(e)));
  // ----- upload -----
  if (hipSetDevice(device) != hipSuccess) return SECPE_EDEVICE_INTERNAL;
  c.tab_bytes = h.size() * sizeof(double);
  HIPCHK(hipMalloc(&c.d_tab, c.tab_bytes));
  HIPCHK(hipMemcpy(c.d_tab, h.data(), c.tab_bytes, hipMemcpyHostToDevice));
  const double* B = c.d_tab;
  c.T.mod = B + o_mod;
  c.T.minv = B + o_minv;
  c.T.psi = B + o_psi;
  c.T.psiq = B + o_psiq;
  c.T.ipsi = B + o_ipsi;
  c.T.ipsiq = B + o_ipsiq;
  c.T.ninv = B + o_ninv;
  c.T.ninvq = B + o_ninvq;
  c.T.cos_hi = B + o_cos_hi;
  c.T.cos_lo = B + o_cos_lo;
  c.T.n_q = n_q;
  c.T.n_p = n_p;
  c.T.log_n = log_n;
  for (auto& kv : doff) c.digits[kv.first] = DigitTable{B + kv.second.cinv, B + kv.second.chat};
  c.md_cinv = B + o_mdc;
  c.md_chat = B + o_mdh;
  c.md_pinv = B + o_mdp;
  c.p_mod_q = B + o_pmq;
  c.rs_tab = B + o_rs;
  c.ytab = B + o_ytab;
  c.rr_cinv = B + o_rrc;
  c.rr_chat = B + o_rrh;
  c.rr_inv = B + o_rri;
  c.md_ytab = B + o_mdy;
  c.rr_ytab = B + o_rry;
  c.crt_tab = B + o_crt;
  HIPCHK(hipEventCreateWithFlags(&c.staging_done, hipEventDisableTiming));
  return 0;
}

void drop_graphs(Ctx& c) {
  if (c.graphs.empty()) return;
  if (c.stream) (void)hipStreamSynchronize(c.stream);
  else (void)hipDeviceSynchronize();
  for (auto& g : c.graphs) {
    if (g.exec) (void)hipGraphExecDestroy(g.exec);
    if (g.graph) (void)hipGraphDestroy(g.graph);
    if (g.arena) (void)hipFree(g.arena);
  }
  c.graphs.clear();
}

void destroy_context(Ctx& c) {
  if (c.stream) (void)hipStreamSynchronize(c.stream);
  else (void)hipDeviceSynchronize();
  drop_graphs(c);
  if (c.d_tab) (void)hipFree(c.d_tab);
  if (c.arena) (void)hipFree(c.arena);
  if (c.staging) (void)hipHostFree(c.staging);
  if (c.client) (void)hipFree(c.client);
  if (c.staging_done) (void)hipEventDestroy(c.staging_done);
  for (hipEvent_t e : c.prof_pool) (void)hipEventDestroy(e);
  c.prof_pool.clear();
  c.d_tab = nullptr;
  c.arena = nullptr;
  c.staging = nullptr;
  c.client = nullptr;
}

// ---------------------------------------------------------------------------
// builder: memory
// ---------------------------------------------------------------------------
Builder::Builder(Ctx& c, char* ws, size_t ws_bytes, char* arena, size_t arena_bytes, bool dry_, SlotPool* pool)
    : C(c), dry(dry_), ws_(ws), ws_bytes_(ws_bytes & ~size_t(255)), arena_(arena), arena_bytes_(arena_bytes) {
  slot_bytes_ = c.ct_bytes();
  pool_ = pool ? pool : &own_pool_;
}

void Builder::note_need() {
  const size_t need = (size_t)pool_->n_slots * slot_bytes_ + scratch_cur_;
  need_max_ = std::max(need_max_, need);
  peak_scratch_ = std::max(peak_scratch_, scratch_cur_);
  if (!dry && need > ws_bytes_) fail(-2, "workspace too small");
}

CT Builder::new_ct(int level, double scale) {
  CT x;
  if (!pool_->free_slots.empty()) {
    x.slot = pool_->free_slots.back();
    pool_->free_slots.pop_back();
  } else {
    x.slot = pool_->n_slots++;
    note_need();
  }
  pool_->live++;
  peak_live_ = std::max(peak_live_, pool_->live);
  x.d = (double*)(ws_ + (size_t)x.slot * slot_bytes_);
  x.level = level;
  x.scale = scale;
  return x;
}

void Builder::free_ct(CT& x) {
  if (x.slot >= 0) {
    pool_->free_slots.push_back(x.slot);
    pool_->live--;
  }
  x.slot = -1;
  x.d = nullptr;
}

double* Builder::scratch(size_t n) {
  n = (n + 31) & ~size_t(31);
  scratch_cur_ += n * sizeof(double);
  note_need();
  // scratch grows downward from the end of the workspace
  return (double*)(ws_ + ws_bytes_ - scratch_cur_);
}

const void* Builder::put_bytes(const void* p, size_t n) {
  size_t off = (blob_.size() + 15) & ~size_t(15);
  blob_.resize(off + n);
  if (n) memcpy(blob_.data() + off, p, n);
  return arena_ + off;
}

const double* Builder::put_residues(int64_t K, int n_limbs) {
  std::vector<double> r(n_limbs);
  for (int t = 0; t < n_limbs; ++t) r[t] = (double)hmod_i64(K, C.mod[t]);
  return put(r);
}

void Builder::push(int kind, int n, int max_y, size_t off, bool inv, int64_t units, int64_t units_shared) {
  // jobs index a grid dimension, which holds at most 65535 workgroups
  if (n > 65535) { fail(-1, "more than 65535 jobs in one launch: split the batch"); return; }
  Cmd c{};
  c.kind = kind;
  c.n = n;
  c.max_y = max_y;
  c.off = off;
  c.inv = inv;
  c.units = units;
  c.units_shared = units_shared < 0 ? units : units_shared;
  cmds_.push_back(c);
  counters[7]++;
}

#define PUSH_JOBS(KIND, V, MAXY, INV, UNITS)                                    \
  do {                                                                          \
    if ((V).empty()) return;                                                    \
    const char* p = (const char*)put(V);                                        \
    push(KIND, (int)(V).size(), MAXY, (size_t)(p - arena_), INV, UNITS);        \
  } while (0)

void Builder::ntt(const std::vector<NttJob>& v, bool inverse, int pass) {
  int my = 0;
  int64_t units = 0;
  for (auto& j : v) {
    my = std::max(my, j.n_limbs);
    const int lo = std::max(0, std::min(j.skip_lo, j.n_limbs)), hi = std::max(lo, std::min(j.skip_hi, j.n_limbs));
    units += j.n_limbs - (hi - lo);
  }
  PUSH_JOBS(pass == 0 ? C_NTT_FIRST : pass == 1 ? C_NTT_SECOND : C_NTT, v, my, inverse, units);
}
void Builder::ew(const std::vector<EwJob>& v) {
  int my = 0;
  int64_t units = 0;
  for (auto& j : v) { my = std::max(my, j.n_limbs); units += j.n_limbs - std::min(j.l_first, j.n_limbs); }
  PUSH_JOBS(C_EW, v, my, false, units);
}
void Builder::modup(const std::vector<ModUpJob>& v) {
  int64_t units = 0;
  for (auto& j : v) units += j.n_ext;
  PUSH_JOBS(C_MODUP, v, 1, false, units);
}
void Builder::modup_col(const std::vector<ModUpJob>& v) {
  int my = 0;
  int64_t units = 0;
  for (auto& j : v) { my = std::max(my, j.n_ext); units += j.n_ext; }
  PUSH_JOBS(C_MODUP_COL, v, my, false, units);
}
void Builder::moddown(const std::vector<ModDownJob>& v) {
  int64_t units = 0;
  for (auto& j : v) units += j.n_chain + C.n_p + (j.first_prime >= 0 ? 1 : 0);
  PUSH_JOBS(C_MODDOWN, v, 1, false, units);
}
void Builder::moddown_col(const std::vector<ModDownJob>& v) {
  int my = 0;
  int64_t units = 0;
  for (auto& j : v) {
    my = std::max(my, j.n_chain);
    units += j.n_chain + C.n_p + (j.first_prime >= 0 ? 1 : 0);
  }
  PUSH_JOBS(C_MODDOWN_COL, v, my, false, units);
}
void Builder::inner(const std::vector<InnerJob>& v, bool row_fused) {
  int my = 0;
  int64_t units = 0, own = 0;
  // a key read by several jobs of the launch: the union of their key limbs,
  // which is the set the highest-level job reads (digit and limb prefixes)
  std::map<const double*, int64_t> key_limbs;
  for (auto& j : v) {
    my = std::max(my, j.n_ext);
    units += (int64_t)j.n_ext * (3 * j.n_digits + 2);
    own += (int64_t)j.n_ext * (j.n_digits + 2);
    int64_t& kl = key_limbs[j.key];
    kl = std::max(kl, (int64_t)2 * j.n_digits * j.n_ext);
  }
  int64_t shared = own;
  for (auto& kv : key_limbs) shared += kv.second;
  if (v.empty()) return;
  const char* p = (const char*)put(v);
  push(row_fused && inner_row_fused(C.T) ? C_INNER_ROW : C_INNER, (int)v.size(), my, (size_t)(p - arena_), false, units,
       shared);
}
void Builder::automorph(const std::vector<AutoJob>& v) {
  int my = 0;
  int64_t units = 0;
  for (auto& j : v) { my = std::max(my, j.n_limbs); units += 2 * j.n_limbs; }
  PUSH_JOBS(C_AUTO, v, my, false, units);
}
void Builder::lift(const std::vector<LiftJob>& v) { PUSH_JOBS(C_LIFT, v, 1, false, 0); }
void Builder::raise(const std::vector<RaiseJob>& v) { PUSH_JOBS(C_RAISE, v, 1, false, 0); }
void Builder::bsgs(const std::vector<BsgsJob>& v) {
  int my = 0;
  for (auto& j : v) my = std::max(my, j.n_limbs);
  PUSH_JOBS(C_BSGS, v, my, false, 0);
}
void Builder::sample(const std::vector<SampleJob>& v) {
  int my = 0;
  for (auto& j : v) my = std::max(my, j.n_limbs);
  PUSH_JOBS(C_SAMPLE, v, my, false, 0);
}
void Builder::intspread(const std::vector<IntSpreadJob>& v) {
  int my = 0;
  for (auto& j : v) my = std::max(my, j.n_limbs);
  PUSH_JOBS(C_INTSPREAD, v, my, false, 0);
}
void Builder::encode(const std::vector<EncodeJob>& v) { PUSH_JOBS(C_ENCODE, v, 1, false, 0); }
void Builder::fft_encode(const std::vector<FftEncJob>& v) {
  if (v.empty()) return;
  const size_t off = (size_t)((const char*)put(v) - arena_);
  const int n = (int)v.size();
  push(C_FFTENC, n, -2, off);
  push(C_FFTENC, n, -1, off);
  for (int st = 0; st <= C.T.log_n; ++st) push(C_FFTENC, n, st, off);
  push(C_FFTENC, n, 1000, off);
}
void Builder::mark() {
  Cmd c{};
  c.kind = C_MARK;
  cmds_.push_back(c);
}
void Builder::decode(const int64_t* m, double* z, int nslots, double inv_scale) {
  Cmd c{};
  c.kind = C_DECODE;
  c.n = nslots;
  c.m = m;
  c.z = z;
  c.inv_scale = inv_scale;
  cmds_.push_back(c);
  counters[7]++;
}

// ---------------------------------------------------------------------------
// submission
// ---------------------------------------------------------------------------
int prof_kind_of(const Cmd& k) {
  switch (k.kind) {
    case C_NTT:
    case C_NTT_FIRST:
    case C_NTT_SECOND: return k.inv ? PROF_NTT_INV : PROF_NTT_FWD;
    case C_EW: return PROF_EW;
    case C_MODUP:
    case C_MODUP_COL: return PROF_MODUP;
    case C_MODDOWN:
    case C_MODDOWN_COL: return PROF_MODDOWN;
    case C_INNER:
    case C_INNER_ROW: return PROF_INNER;
    case C_AUTO: return PROF_AUTO;
    default: return -1;
  }
}

static hipEvent_t prof_event(Ctx& c) {
  if (c.prof_used == c.prof_pool.size()) {
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    c.prof_pool.push_back(e);
  }
  return c.prof_pool[c.prof_used++];
}

void launch_cmds(Ctx& c, const std::vector<Cmd>& cmds, char* arena) {
  const DevTables& T = c.T;
  hipStream_t s = c.stream;
  // segment profiler: an event at the start, at every mark and at the end
  const bool seg = c.prof_kind == PROF_SEGMENTS;
  if (seg) {
    hipEvent_t e = prof_event(c);
    if (e) (void)hipEventRecord(e, s);
  }
  for (const Cmd& k : cmds) {
    if (k.kind == C_MARK) {
      if (seg) {
        hipEvent_t e = prof_event(c);
        if (e) (void)hipEventRecord(e, s);
      }
      continue;
    }
    const void* j = arena + k.off;
    if ((k.kind == C_NTT || k.kind == C_NTT_FIRST || k.kind == C_NTT_SECOND) && ntt_pass_count(T) == 2) {
      // Two-pass NTT, issued in groups of jobs whose data fits ntt_chunk_bytes
      // so the intermediate between the passes can stay in the Infinity
      // Cache.  The pass profilers bracket each launch of their pass.
      const int pass_prof = c.prof_kind == PROF_NTT_FWD_COL && !k.inv ? 0
                            : c.prof_kind == PROF_NTT_FWD_ROW && !k.inv ? 1 : -1;
      const bool whole_prof = c.prof_kind >= 0 && prof_kind_of(k) == c.prof_kind;
      const size_t per_job = (size_t)std::max(1, k.max_y) * c.N * sizeof(double);
      int chunk = k.n;
      if (c.ntt_chunk_bytes > 0) chunk = (int)std::max<size_t>(1, c.ntt_chunk_bytes / per_job);
      hipEvent_t w0 = whole_prof ? prof_event(c) : nullptr;
      if (w0) (void)hipEventRecord(w0, s);
      const int p_lo = k.kind == C_NTT_SECOND ? 1 : 0, p_hi = k.kind == C_NTT_FIRST ? 1 : 2;
      // a single-pass launch counts as half of its limb transforms
      if (whole_prof) {
        c.prof_launches++;
        c.prof_units += p_hi - p_lo == 2 ? k.units : k.units / 2;
        c.prof_units_shared += p_hi - p_lo == 2 ? k.units_shared : k.units_shared / 2;
      }
      const NttJob* jobs = (const NttJob*)j;
      for (int j0 = 0; j0 < k.n; j0 += chunk) {
        const int nj = std::min(chunk, k.n - j0);
        for (int pass = p_lo; pass < p_hi; ++pass) {
          hipEvent_t e0 = pass == pass_prof ? prof_event(c) : nullptr;
          if (e0) {
            (void)hipEventRecord(e0, s);
            c.prof_launches++;
          }
          launch_ntt_pass(T, k.inv, jobs + j0, nj, k.max_y, pass, s, c.ntt_tiles);
          if (e0) {
            hipEvent_t e1 = prof_event(c);
            if (e1) (void)hipEventRecord(e1, s);
          }
        }
      }
      if (pass_prof >= p_lo && pass_prof < p_hi) {
        c.prof_units += k.units;
        c.prof_units_shared += k.units_shared;
      }
      if (w0) {
        hipEvent_t w1 = prof_event(c);
        if (w1) (void)hipEventRecord(w1, s);
      }
      continue;
    }
    const bool prof = c.prof_kind >= 0 && prof_kind_of(k) == c.prof_kind;
    if (prof) {
      hipEvent_t e = prof_event(c);
      if (e) (void)hipEventRecord(e, s);
      c.prof_launches++;
      c.prof_units += k.units;
      c.prof_units_shared += k.units_shared;
    }
    switch (k.kind) {
      case C_NTT: launch_ntt(T, k.inv, (const NttJob*)j, k.n, k.max_y, s, c.ntt_tiles); break;
      case C_NTT_FIRST: launch_ntt_pass(T, k.inv, (const NttJob*)j, k.n, k.max_y, 0, s, c.ntt_tiles); break;
      case C_NTT_SECOND: launch_ntt_pass(T, k.inv, (const NttJob*)j, k.n, k.max_y, 1, s, c.ntt_tiles); break;
      case C_EW: launch_ew(T, (const EwJob*)j, k.n, k.max_y, s); break;
      case C_MODUP: launch_modup(T, (const ModUpJob*)j, k.n, s); break;
      case C_MODUP_COL: launch_modup_col(T, (const ModUpJob*)j, k.n, k.max_y, c.modup_eg, s); break;
      case C_MODDOWN: launch_moddown_conv(T, (const ModDownJob*)j, k.n, s); break;
      case C_MODDOWN_COL: launch_moddown_col(T, (const ModDownJob*)j, k.n, k.max_y, c.moddown_eg, s); break;
      case C_INNER: launch_inner(T, (const InnerJob*)j, k.n, k.max_y, s); break;
      case C_INNER_ROW: launch_inner_row(T, (const InnerJob*)j, k.n, k.max_y, s); break;
      case C_AUTO: launch_automorph(T, (const AutoJob*)j, k.n, k.max_y, s); break;
      case C_LIFT: launch_lift(T, (const LiftJob*)j, k.n, c.crt_tab, c.q0inv_q1, s); break;
      case C_RAISE: launch_raise(T, (const RaiseJob*)j, k.n, s); break;
      case C_BSGS: launch_bsgs(T, (const BsgsJob*)j, k.n, k.max_y, s); break;
      case C_SAMPLE: launch_sample(T, (const SampleJob*)j, k.n, k.max_y, s); break;
      case C_INTSPREAD: launch_int_spread(T, (const IntSpreadJob*)j, k.n, k.max_y, s); break;
      case C_ENCODE: launch_encode(T, (const EncodeJob*)j, k.n, s); break;
      case C_FFTENC: launch_fft_enc(T, (const FftEncJob*)j, k.n, k.max_y, s); break;
      case C_DECODE: launch_decode(T, k.m, k.z, k.n, k.inv_scale, s); break;
      default: break;
    }
    if (prof) {
      hipEvent_t e = prof_event(c);
      if (e) (void)hipEventRecord(e, s);
    }
  }
  if (seg) {
    hipEvent_t e = prof_event(c);
    if (e) (void)hipEventRecord(e, s);
    c.prof_launches++;
  }
}

int submit(Ctx& c, Builder& b, char* arena, size_t arena_bytes, bool may_allocate) {
  const size_t n = b.blob_.size();
  if (n > arena_bytes) return -2;
  if (n) {
    if (c.staging_bytes < n && !may_allocate) return -2;
    if (c.staging_bytes < n) {
      if (c.staging) {
        (void)hipEventSynchronize(c.staging_done);
        (void)hipHostFree(c.staging);
      }
      c.staging_bytes = std::max(n, c.staging_bytes * 2);
      if (hipHostMalloc((void**)&c.staging, c.staging_bytes, hipHostMallocDefault) != hipSuccess) {
        c.staging = nullptr;
        c.staging_bytes = 0;
        return -5;
      }
    } else {
      (void)hipEventSynchronize(c.staging_done);
    }
    memcpy(c.staging, b.blob_.data(), n);
    if (hipMemcpyAsync(arena, c.staging, n, hipMemcpyHostToDevice, c.stream) != hipSuccess) return -5;
    (void)hipEventRecord(c.staging_done, c.stream);
  }
  launch_cmds(c, b.cmds_, arena);
  if (hipGetLastError() != hipSuccess) return -5;
  return 0;
}

// ---------------------------------------------------------------------------
// key switching (hybrid, digits of alpha chain primes)
//   ModUp each digit -> inner product with the key over Q_l u P -> ModDown
// ---------------------------------------------------------------------------
// first half, shared by key switching and the merged relinearise + rescale:
// the accumulator acc_w over Q_l u P (NTT domain) with acc0 + acc1 s' = P d s + small
void Builder::ks_front(const std::vector<KsItem>& items, std::vector<KsTmp>& tmp, bool merged) {
  const int N = C.N, alpha = C.alpha, n_p = C.n_p;
  const bool fused = inner_row_fused(C.T);
  tmp.resize(items.size());
  std::vector<NttJob> j_inv, j_fwd_ext;
  std::vector<ModUpJob> j_up;
  std::vector<InnerJob> j_in;
  for (size_t i = 0; i < items.size(); ++i) {
    const KsItem& it = items[i];
    const int l = it.level, nc = l + 1, n_ext = nc + n_p;
    const int nd = (nc + alpha - 1) / alpha;
    KsTmp& t = tmp[i];
    t.n_ext = n_ext;
    t.dcoef = scratch((size_t)nc * N);
    t.ext = scratch((size_t)nd * n_ext * N);
    t.acc = scratch((size_t)2 * n_ext * N);
    NttJob ji{it.d, t.dcoef, nc, nc, 0, 0};
    ji.sq = it.square ? 1 : 0;
    // fused path: the inverse transform leaves the ModUp digits y_t = [x_t (D_j/q_t)^-1]
    if (fused) ji.ek = C.ytab + (size_t)l * C.n_q;
    j_inv.push_back(ji);
    for (int j = 0; j < nd; ++j) {
      const int lo = j * alpha, hi = std::min((j + 1) * alpha, nc);
      const DigitTable& dt = C.digits.at({lo, hi - lo});
      double* e = t.ext + (size_t)j * n_ext * N;
      j_up.push_back(ModUpJob{t.dcoef, e, dt.cinv, dt.chat, lo, hi, nc, n_ext});
      j_fwd_ext.push_back(NttJob{e, e, n_ext, nc, lo, hi});
    }
    InnerJob in{it.d, t.ext, it.key, t.acc, it.top0, it.top1, C.p_mod_q, nc, n_ext, nd, alpha};
    // algorithmic-byte accounting: ciphertext limbs in and out
    ks_alg_limbs += 3 * (int64_t)nc;
    in.inv_from = fused ? (merged ? l : l + 1) : n_ext;
    in.d_square = it.square ? 1 : 0;
    j_in.push_back(in);
  }
  // ... and each distinct key once for the launch (its highest-level reader)
  {
    std::map<const double*, int64_t> kl;
    for (const KsItem& it : items) {
      const int nc = it.level + 1, nd = (nc + alpha - 1) / alpha;
      int64_t& v = kl[it.key];
      v = std::max(v, (int64_t)2 * nd * (nc + n_p));
    }
    for (auto& kv : kl) ks_alg_limbs += kv.second;
  }
  ntt(j_inv, true);
  if (fused) {
    // ModUp + column pass in one kernel; the row pass runs inside the inner product
    modup_col(j_up);
  } else {
    modup(j_up);
    ntt(j_fwd_ext, false);
  }
  inner(j_in);
}

// key switching (hybrid): front half, then ModDown by P
void Builder::key_switch(const std::vector<KsItem>& items) {
  std::vector<KsTmp> tmp;
  ks_front(items, tmp, false);
  ks_back(items, tmp, inner_row_fused(C.T));
}

void Builder::ks_back(const std::vector<KsItem>& items, const std::vector<KsTmp>& tmp, bool first_pass_done) {
  const int N = C.N, n_p = C.n_p;
  std::vector<NttJob> j_inv_acc, j_fwd_conv;
  std::vector<ModDownJob> j_down;
  for (size_t i = 0; i < items.size(); ++i) {
    const KsItem& it = items[i];
    const int nc = it.level + 1, n_ext = tmp[i].n_ext;
    double* acc = tmp[i].acc;
    double* conv = scratch((size_t)2 * nc * N);
    for (int w = 0; w < 2; ++w) {
      double* aw = acc + (size_t)w * n_ext * N;
      double* sp = aw + (size_t)nc * N;
      // the inverse transform's last pass applies (P/p_k)^-1 for the conversion
      NttJob ji{sp, sp, n_p, 0, 0, 0};
      ji.ek = C.md_ytab;
      ji.centre = 1;
      j_inv_acc.push_back(ji);
      double* cv = conv + (size_t)w * nc * N;
      j_down.push_back(ModDownJob{sp, cv, nullptr, C.md_chat, nc, -1});
      // out_w = base_w + (acc_w - NTT(conv_w)) P^-1, fused into the transform
      NttJob f{cv, cv, nc, nc, 0, 0};
      f.epi = EPI_MODDOWN;
      f.eb = aw;
      f.ebase = w ? it.base1 : it.base0;
      f.eout = w ? it.out1 : it.out0;
      f.ek = C.md_pinv;
      j_fwd_conv.push_back(f);
    }
  }
  ntt(j_inv_acc, true, first_pass_done ? 1 : -1);
  if (inner_row_fused(C.T)) {
    // conversion + column pass in one kernel; the row pass carries the combine
    moddown_col(j_down);
    ntt(j_fwd_conv, false, 1);
  } else {
    moddown(j_down);
    ntt(j_fwd_conv, false);
  }
  counters[3] += (int64_t)items.size();
}

Builder::Hoisted Builder::hoist(const std::vector<CT>& in) {
  const int N = C.N, alpha = C.alpha, n_p = C.n_p;
  const bool fused = inner_row_fused(C.T);
  Hoisted h;
  h.in = in;
  for (const CT& x : in) {
    const int nc = x.level + 1, nd = (nc + alpha - 1) / alpha;
    h.ext.push_back(scratch((size_t)nd * (nc + n_p) * N));
  }
  const size_t mark = scratch_mark();
  std::vector<NttJob> j_inv, j_fwd_ext;
  std::vector<ModUpJob> j_up;
  for (size_t i = 0; i < in.size(); ++i) {
    const CT& x = in[i];
    const int l = x.level, nc = l + 1, n_ext = nc + n_p, nd = (nc + alpha - 1) / alpha;
    double* dcoef = scratch((size_t)nc * N);
    NttJob ji{c1(x), dcoef, nc, nc, 0, 0};
    if (fused) ji.ek = C.ytab + (size_t)l * C.n_q;
    j_inv.push_back(ji);
    for (int j = 0; j < nd; ++j) {
      const int lo = j * alpha, hi = std::min((j + 1) * alpha, nc);
      const DigitTable& dt = C.digits.at({lo, hi - lo});
      double* e = h.ext[i] + (size_t)j * n_ext * N;
      j_up.push_back(ModUpJob{dcoef, e, dt.cinv, dt.chat, lo, hi, nc, n_ext});
      j_fwd_ext.push_back(NttJob{e, e, n_ext, nc, lo, hi});
    }
  }
  ntt(j_inv, true);
  if (fused) {
    // ModUp + column pass, then the row pass on its own: the automorphism
    // needs each raised limb fully transformed
    modup_col(j_up);
    ntt(j_fwd_ext, false, 1);
  } else {
    modup(j_up);
    ntt(j_fwd_ext, false);
  }
  scratch_release(mark);
  return h;
}

// ext limbs on a digit's own primes are never written (the inner product
// reads those from d); the automorphism permutes them along unread.
// With a permuted key (keys_perm) the raised digits are not permuted at all:
// sum_j X^g(ext_j) key_j = X^g(sum_j ext_j X^(g^-1)(key_j)), and the ModDown
// commutes with X -> X^g residue for residue (the inverse and forward
// transforms, the centred conversion and the division by P all do), so the
// inner product of the unpermuted digits with the permuted key, the ModDown
// onto c0, and one permutation of the two result polynomials give the same
// residues as permuting the digits first.
std::vector<CT> Builder::rotate_hoisted(const Hoisted& h, const std::vector<int64_t>& steps) {
  const int N = C.N, alpha = C.alpha, n_p = C.n_p;
  const size_t mark = scratch_mark();
  std::vector<CT> out;
  std::vector<AutoJob> j_a, j_post;
  std::vector<InnerJob> j_in;
  std::vector<KsItem> ks;
  std::vector<KsTmp> tmp;
  std::map<const double*, int64_t> key_limbs;
  for (int64_t st : steps) {
    const uint64_t g = C.galois(st);
    const double* gk = nullptr;
    const double* pk = nullptr;
    if (g != 1) {
      auto it = C.keys.find(g);
      gk = it != C.keys.end() ? it->second : (dry ? C.T.mod : nullptr);
      if (!gk) { fail(-4, "no Galois key for rotation " + std::to_string(st)); return {}; }
      auto pit = C.keys_perm.find(g);
      if (pit != C.keys_perm.end()) pk = pit->second;
    }
    for (size_t i = 0; i < h.in.size(); ++i) {
      const CT& x = h.in[i];
      const int nc = x.level + 1, n_ext = nc + n_p, nd = (nc + alpha - 1) / alpha;
      CT o = new_ct(x.level, x.scale);
      if (g == 1) {
        EwJob e{};
        e.o0 = c0(o); e.o1 = c1(o); e.a0 = c0(x); e.a1 = c1(x);
        e.n_limbs = nc; e.n_chain = nc; e.op = EW_COPY;
        ew({e});
        out.push_back(o);
        continue;
      }
      double* acc = scratch((size_t)2 * n_ext * N);
      if (pk) {
        double* r = scratch((size_t)2 * nc * N);
        InnerJob in{c1(x), h.ext[i], pk, acc, nullptr, nullptr, C.p_mod_q, nc, n_ext, nd, alpha};
        in.inv_from = n_ext;
        in.d_square = 0;
        j_in.push_back(in);
        ks.push_back(KsItem{c1(x), x.level, pk, c0(x), nullptr, r, r + (size_t)nc * N, nullptr, nullptr, false});
        tmp.push_back(KsTmp{nullptr, h.ext[i], acc, n_ext});
        j_post.push_back(AutoJob{r, c0(o), nc, nc, (uint32_t)g, 0});
        j_post.push_back(AutoJob{r + (size_t)nc * N, c1(o), nc, nc, (uint32_t)g, 0});
      } else {
        double* d = scratch((size_t)nc * N);
        double* es = scratch((size_t)nd * n_ext * N);
        j_a.push_back(AutoJob{c0(x), c0(o), nc, nc, (uint32_t)g, 0});
        j_a.push_back(AutoJob{c1(x), d, nc, nc, (uint32_t)g, 0});
        j_a.push_back(AutoJob{h.ext[i], es, nd * n_ext, nd * n_ext, (uint32_t)g, 0});
        InnerJob in{d, es, gk, acc, nullptr, nullptr, C.p_mod_q, nc, n_ext, nd, alpha};
        in.inv_from = n_ext;
        in.d_square = 0;
        j_in.push_back(in);
        ks.push_back(KsItem{d, x.level, gk, c0(o), nullptr, c0(o), c1(o), nullptr, nullptr, false});
        tmp.push_back(KsTmp{nullptr, es, acc, n_ext});
      }
      // algorithmic-byte accounting: ciphertext limbs in and out, each key once
      ks_alg_limbs += 3 * (int64_t)nc;
      int64_t& kl = key_limbs[gk];
      kl = std::max(kl, (int64_t)2 * nd * n_ext);
      out.push_back(o);
    }
  }
  for (auto& kv : key_limbs) ks_alg_limbs += kv.second;
  if (!ks.empty()) {
    automorph(j_a);
    inner(j_in, false);
    ks_back(ks, tmp, false);
    automorph(j_post);
    counters[1] += (int64_t)ks.size();
  }
  scratch_release(mark);
  return out;
}

// merged relinearise + rescale of degree-2 ciphertexts (d0, d1, d2) at level l:
// y_w = P d_w + acc_w over Q_l u P, divided by B = P q_l with a centred base
// conversion from {q_l} u P: out_w = (y_w - Conv_B(y_w)) B^-1 on limbs 0..l-1
std::vector<CT> Builder::relin_rescale(const std::vector<Deg2>& xs) {
  const int N = C.N, n_p = C.n_p, n_q = C.n_q, nb = n_p + 1;
  auto kit = C.keys.find(0);
  const double* rk = kit != C.keys.end() ? kit->second : (dry ? C.T.mod : nullptr);
  if (!rk) { fail(-4, "no relinearisation key"); return {}; }
  std::vector<KsItem> items;
  for (const Deg2& x : xs) {
    if (x.level < 1) { fail(-3, "relinearise-and-rescale at level 0"); return {}; }
    if (x.sq0) {
      if (!inner_row_fused(C.T)) { fail(-1, "fused squares need the two-pass NTT"); return {}; }
      items.push_back(KsItem{x.sq1, x.level, rk, nullptr, nullptr, nullptr, nullptr, x.sq0, x.sq1, true});
    } else {
      items.push_back(KsItem{x.d2, x.level, rk, nullptr, nullptr, nullptr, nullptr, x.d0, x.d1, false});
    }
  }
  std::vector<KsTmp> tmp;
  ks_front(items, tmp, true);
  std::vector<CT> out;
  std::vector<NttJob> j_inv_acc, j_fwd_conv;
  std::vector<ModDownJob> j_conv;
  for (size_t i = 0; i < xs.size(); ++i) {
    const Deg2& x = xs[i];
    const int l = x.level, nc = l + 1, n_ext = tmp[i].n_ext;
    double* acc = tmp[i].acc;
    double* conv = scratch((size_t)2 * l * N);
    CT o = new_ct(l - 1, x.scale / (double)C.mod[l]);
    for (int w = 0; w < 2; ++w) {
      double* aw = acc + (size_t)w * n_ext * N;
      // limbs l .. l+n_p of the extended basis: q_l, then the special primes
      // (its last pass also applies (B/b)^-1 for the conversion)
      NttJob ji{aw, aw, n_ext, nc, 0, l};
      ji.ek = C.rr_ytab + (size_t)l * (n_q + n_p);
      ji.centre = 1;
      j_inv_acc.push_back(ji);
      double* cv = conv + (size_t)w * l * N;
      j_conv.push_back(ModDownJob{aw + (size_t)l * N, cv, nullptr, C.rr_chat + (size_t)l * n_q * nb, l, l});
      // out_w = (P d_w + acc_w - NTT(conv_w)) (P q_l)^-1, fused into the transform
      NttJob f{cv, cv, l, l, 0, 0};
      f.epi = EPI_RRCOMB;
      if (x.sq0) {
        // d0 = a0^2, d1 = 2 a0 a1 of the square, formed in the epilogue
        f.ea = x.sq0;
        f.ebase = x.sq1;
        f.sq = w ? 2 : 1;
      } else {
        f.ea = w ? x.d1 : x.d0;
      }
      f.eb = aw;
      f.eout = w ? c1(o) : c0(o);
      f.ek = C.rr_inv + (size_t)l * n_q;
      f.ek2 = C.p_mod_q;
      j_fwd_conv.push_back(f);
    }
    out.push_back(o);
  }
  // (fused: the first inverse pass already ran inside the inner product)
  ntt(j_inv_acc, true, inner_row_fused(C.T) ? 1 : -1);
  if (inner_row_fused(C.T)) {
    moddown_col(j_conv);
    ntt(j_fwd_conv, false, 1);
  } else {
    moddown(j_conv);
    ntt(j_fwd_conv, false);
  }
  counters[2] += (int64_t)xs.size();
  counters[3] += (int64_t)xs.size();
  return out;
}

// degree-2 sums: for each item, x.a (x) x.b [+ x.c (x) x.e] [+ x.f] at the
// lowest level among the operands
static int64_t const_for(double v, double target, double q, double s, bool rescale, bool& ok);

std::vector<Builder::Deg2> Builder::tensor2(const std::vector<TensorItem>& v) {
  const int N = C.N;
  std::vector<Deg2> out;
  std::vector<EwJob> j;
  for (const TensorItem& it : v) {
    int l = std::min(it.a.level, it.b.level);
    double sc = it.a.scale * it.b.scale;
    if (it.has_ce) {
      l = std::min(l, std::min(it.c.level, it.e.level));
      const double s2 = it.c.scale * it.e.scale;
      if (fabs(sc - s2) > 1e-9 * fabs(sc)) { fail(-1, "scale mismatch in degree-2 sum"); return {}; }
    }
    if (it.has_f) {
      if (it.f.level < l) { fail(-1, "addend below the product level"); return {}; }
      if (fabs(sc - it.f.scale) > 1e-9 * fabs(sc)) { fail(-1, "scale mismatch in degree-2 sum"); return {}; }
    }
    if (it.has_fl) {
      const LinItem& L = it.fl;
      if (L.has_b && L.b.level != L.a.level) { fail(-1, "lincomb: level mismatch"); return {}; }
      if (L.a.level < l) { fail(-1, "addend below the product level"); return {}; }
      if (fabs(sc - L.target) > 1e-9 * fabs(sc)) { fail(-1, "scale mismatch in degree-2 sum"); return {}; }
    }
    Deg2 d{};
    d.level = l;
    d.scale = sc;
    d.d0 = scratch((size_t)(l + 1) * N);
    d.d1 = scratch((size_t)(l + 1) * N);
    d.d2 = scratch((size_t)(l + 1) * N);
    EwJob e{};
    e.o0 = d.d0; e.o1 = d.d1; e.o2 = d.d2;
    e.a0 = c0(it.a); e.a1 = c1(it.a);
    e.b0 = c0(it.b); e.b1 = c1(it.b);
    if (it.has_ce) { e.c0 = c0(it.c); e.c1 = c1(it.c); e.e0 = c0(it.e); e.e1 = c1(it.e); }
    if (it.has_f) { e.f0 = c0(it.f); e.f1 = c1(it.f); }
    if (it.has_fl) {
      // the constants EW_LIN2 would use for the same combination (unrescaled)
      const LinItem& L = it.fl;
      bool ok1 = true, ok2 = true;
      const int64_t Ka = const_for(L.va, L.target, 0.0, L.a.scale, false, ok1);
      const int64_t Kb = L.has_b ? const_for(L.vb, L.target, 0.0, L.b.scale, false, ok2) : 0;
      if (!ok1 || !ok2) { fail(-1, "constant does not fit 64 bits"); return {}; }
      e.f0 = c0(L.a); e.f1 = c1(L.a);
      e.k = put_residues(Ka, l + 1);
      if (L.has_b) {
        e.g0 = c0(L.b); e.g1 = c1(L.b);
        e.k2 = put_residues(Kb, l + 1);
      }
    }
    e.n_limbs = l + 1; e.n_chain = l + 1;
    e.op = EW_TENSOR2;
    j.push_back(e);
    out.push_back(d);
  }
  ew(j);
  return out;
}

// rescale by the top prime q_l: c_i <- (c_i - [c_l]centred) * q_l^-1  (in place)
void Builder::rescale(std::vector<CT>& xs) { rescale(xs, nullptr); }

void Builder::rescale(std::vector<CT>& xs, const std::vector<LinSrc>* lin) {
  const int N = C.N;
  std::vector<NttJob> j_top, j_fwd;
  for (size_t xi = 0; xi < xs.size(); ++xi) {
    CT& x = xs[xi];
    const int l = x.level;
    if (l < 1) { fail(-3, "rescale below level 0"); return; }
    double* top = scratch(2 * (size_t)N);
    double* spr = scratch(2 * (size_t)l * N);
    for (int w = 0; w < 2; ++w) {
      double* cw = w ? c1(x) : c0(x);
      double* tw = top + (size_t)w * N;
      // transform only limb l: limbs [0, l) skipped; dst shifted so limb l lands in tw
      j_top.push_back(NttJob{cw, tw - (size_t)l * N, l + 1, l + 1, 0, l});
      // forward NTT of the centred top limb reduced mod each q_i (fused
      // spread), then c_i <- (c_i - that) q_l^-1 in place (fused epilogue)
      NttJob f{tw, spr + (size_t)w * l * N, l, l, 0, 0};
      f.spread_from = l + 1;
      f.epi = EPI_RESCALE;
      f.ea = cw;
      f.eout = cw;
      f.ek = C.rs_tab + (size_t)l * C.n_q;
      if (lin) {
        // limbs below l of the combination are formed from its sources here
        const LinSrc& ls = (*lin)[xi];
        f.epi = EPI_LINRS;
        f.ea = w ? ls.a1 : ls.a0;
        f.eb = w ? ls.b1 : ls.b0;
        f.ek2 = ls.ka;
        f.ek3 = ls.kb;
      }
      j_fwd.push_back(f);
    }
    x.scale = x.scale / (double)C.mod[l];
    x.level = l - 1;
  }
  ntt(j_top, true);
  ntt(j_fwd, false);
}

std::vector<CT> Builder::mul_relin(const std::vector<std::pair<CT, CT>>& ab, bool do_rescale) {
  const int N = C.N;
  const size_t mark = scratch_mark();
  if (do_rescale) {
    // squares at two-pass sizes skip the tensor product: the kernels that
    // read d0, d1, d2 form them from the operand
    const bool fuse_sq = inner_row_fused(C.T);
    std::vector<TensorItem> ti;
    std::vector<int> where(ab.size(), -1);
    for (size_t i = 0; i < ab.size(); ++i) {
      const auto& p = ab[i];
      if (fuse_sq && p.first.d == p.second.d && p.first.level == p.second.level) continue;
      TensorItem t{};
      t.a = p.first;
      t.b = p.second;
      where[i] = (int)ti.size();
      ti.push_back(t);
    }
    std::vector<Deg2> dt = tensor2(ti);
    if (err_code) return {};
    std::vector<Deg2> d;
    for (size_t i = 0; i < ab.size(); ++i) {
      if (where[i] >= 0) {
        d.push_back(dt[where[i]]);
        continue;
      }
      Deg2 q{};
      q.level = ab[i].first.level;
      q.scale = ab[i].first.scale * ab[i].second.scale;
      q.sq0 = c0(ab[i].first);
      q.sq1 = c1(ab[i].first);
      d.push_back(q);
    }
    std::vector<CT> out = relin_rescale(d);
    if (err_code) return {};
    scratch_release(mark);
    return out;
  }
  auto it = C.keys.find(0);
  const double* rk = it != C.keys.end() ? it->second : (dry ? C.T.mod : nullptr);
  if (!rk) { fail(-4, "no relinearisation key"); return {}; }
  std::vector<CT> out;
  std::vector<EwJob> j_t;
  std::vector<KsItem> ks;
  for (auto& p : ab) {
    const int l = std::min(p.first.level, p.second.level);
    CT o = new_ct(l, p.first.scale * p.second.scale);
    double* d2 = scratch((size_t)(l + 1) * N);
    EwJob e{};
    e.o0 = c0(o);
    e.o1 = c1(o);
    e.o2 = d2;
    e.a0 = c0(p.first);
    e.a1 = c1(p.first);
    e.b0 = c0(p.second);
    e.b1 = c1(p.second);
    e.n_limbs = l + 1;
    e.n_chain = l + 1;
    e.op = EW_TENSOR;
    j_t.push_back(e);
    ks.push_back(KsItem{d2, l, rk, c0(o), c1(o), c0(o), c1(o), nullptr, nullptr, false});
    out.push_back(o);
  }
  ew(j_t);
  key_switch(ks);
  counters[2] += (int64_t)ab.size();
  if (err_code) return {};
  scratch_release(mark);
  return out;
}

std::vector<CT> Builder::rotate(const std::vector<CT>& in, const std::vector<int64_t>& steps) {
  const int N = C.N;
  const size_t mark = scratch_mark();
  std::vector<CT> out;
  std::vector<AutoJob> j_a;
  std::vector<KsItem> ks;
  for (size_t i = 0; i < in.size(); ++i) {
    const CT& x = in[i];
    const uint64_t g = C.galois(steps[i]);
    CT o = new_ct(x.level, x.scale);
    const int nl = x.level + 1;
    if (g == 1) {
      EwJob e{};
      e.o0 = c0(o); e.o1 = c1(o); e.a0 = c0(x); e.a1 = c1(x);
      e.n_limbs = nl; e.n_chain = nl; e.op = EW_COPY;
      ew({e});
      out.push_back(o);
      continue;
    }
    auto it = C.keys.find(g);
    const double* gk = it != C.keys.end() ? it->second : (dry ? C.T.mod : nullptr);
    if (!gk) { fail(-4, "no Galois key for rotation " + std::to_string(steps[i])); return {}; }
    double* d = scratch((size_t)nl * N);
    j_a.push_back(AutoJob{c0(x), c0(o), nl, nl, (uint32_t)g, 0});
    j_a.push_back(AutoJob{c1(x), d, nl, nl, (uint32_t)g, 0});
    ks.push_back(KsItem{d, x.level, gk, c0(o), nullptr, c0(o), c1(o), nullptr, nullptr, false});
    out.push_back(o);
  }
  automorph(j_a);
  key_switch(ks);
  counters[1] += (int64_t)ks.size();
  scratch_release(mark);
  return out;
}

std::vector<CT> Builder::add(const std::vector<std::pair<CT, CT>>& ab, bool sub) {
  std::vector<CT> out;
  std::vector<EwJob> j;
  for (auto& p : ab) {
    const double sa = p.first.scale, sb = p.second.scale;
    if (fabs(sa - sb) > 1e-9 * fabs(sa)) { fail(-1, "scale mismatch in addition"); return {}; }
    const int l = std::min(p.first.level, p.second.level);
    CT o = new_ct(l, sa);
    EwJob e{};
    e.o0 = c0(o); e.o1 = c1(o);
    e.a0 = c0(p.first); e.a1 = c1(p.first);
    e.b0 = c0(p.second); e.b1 = c1(p.second);
    e.n_limbs = l + 1; e.n_chain = l + 1;
    e.op = sub ? EW_SUB : EW_ADD;
    j.push_back(e);
    out.push_back(o);
  }
  ew(j);
  return out;
}

void Builder::add_sub(const std::vector<std::pair<CT, CT>>& ab, std::vector<CT>& diff, std::vector<CT>& sum) {
  diff.clear();
  sum.clear();
  std::vector<EwJob> j;
  for (auto& p : ab) {
    const double sa = p.first.scale, sb = p.second.scale;
    if (fabs(sa - sb) > 1e-9 * fabs(sa)) { fail(-1, "scale mismatch in addition"); return; }
    const int l = std::min(p.first.level, p.second.level);
    CT d = new_ct(l, sa);
    CT s = new_ct(l, sa);
    for (int w = 0; w < 2; ++w) {
      EwJob e{};
      e.o0 = w ? c1(d) : c0(d);
      e.o1 = w ? c1(s) : c0(s);
      e.a0 = w ? c1(p.first) : c0(p.first);
      e.b0 = w ? c1(p.second) : c0(p.second);
      e.n_limbs = l + 1; e.n_chain = l + 1;
      e.op = EW_ADDSUB;
      j.push_back(e);
    }
    diff.push_back(d);
    sum.push_back(s);
  }
  ew(j);
}

std::vector<CT> Builder::add_const(const std::vector<CT>& in, const std::vector<double>& v) {
  std::vector<CT> out;
  std::vector<EwJob> j;
  for (size_t i = 0; i < in.size(); ++i) {
    const CT& x = in[i];
    double kf = v[i] * x.scale;
    const int64_t K = llround(kf);
    CT o = new_ct(x.level, x.scale);
    EwJob e{};
    e.o0 = c0(o); e.o1 = c1(o); e.a0 = c0(x); e.a1 = c1(x);
    e.k = put_residues(K, x.level + 1);
    e.n_limbs = x.level + 1; e.n_chain = x.level + 1;
    e.op = EW_ADD_CONST;
    j.push_back(e);
    out.push_back(o);
  }
  ew(j);
  return out;
}

// integer constant taking value v at scale s to scale T: llround(v T q / s)
// when a rescale by q follows, llround(v T / s) when none does
static int64_t const_for(double v, double target, double q, double s, bool rescale, bool& ok) {
  double k = v * target;
  if (rescale) k = k * q;
  k = k / s;
  ok = fabs(k) < 9.2e18;
  return ok ? llround(k) : 0;
}

// K_a a + K_b b with constants chosen so the result carries scale T: rescaled
// once, or left at the operands' level when 'rescale' is false
std::vector<CT> Builder::lincomb(const std::vector<LinItem>& v, bool do_rescale) {
  std::vector<CT> out;
  std::vector<EwJob> j;
  std::vector<LinSrc> lin;
  for (const LinItem& it : v) {
    const CT& x = it.a;
    if (it.has_b && it.b.level != x.level) { fail(-1, "lincomb: level mismatch"); return {}; }
    const double ql = (double)C.mod[x.level];
    bool ok1 = true, ok2 = true;
    const int64_t Ka = const_for(it.va, it.target, ql, x.scale, do_rescale, ok1);
    const int64_t Kb = it.has_b ? const_for(it.vb, it.target, ql, it.b.scale, do_rescale, ok2) : 0;
    if (!ok1 || !ok2) { fail(-1, "constant does not fit 64 bits"); return {}; }
    CT o = new_ct(x.level, it.target);
    EwJob e{};
    e.o0 = c0(o); e.o1 = c1(o); e.a0 = c0(x); e.a1 = c1(x);
    e.k = put_residues(Ka, x.level + 1);
    if (it.has_b) {
      e.b0 = c0(it.b); e.b1 = c1(it.b);
      e.k2 = put_residues(Kb, x.level + 1);
    }
    e.n_limbs = x.level + 1; e.n_chain = x.level + 1;
    e.op = EW_LIN2;
    if (do_rescale) {
      // only the top limb is formed here: the rescale's forward transform
      // forms the others in its epilogue, from the same sources
      e.l_first = x.level;
      lin.push_back(LinSrc{e.a0, e.a1, e.b0, e.b1, e.k, e.k2});
    }
    j.push_back(e);
    out.push_back(o);
  }
  ew(j);
  if (do_rescale) {
    const size_t mark = scratch_mark();
    rescale(out, &lin);
    scratch_release(mark);
    if (err_code) return {};
    for (size_t i = 0; i < out.size(); ++i) out[i].scale = v[i].target;
  }
  return out;
}

// constant product with exact target scale: K = llround(v T q_l / s), rescale, scale := T
std::vector<CT> Builder::mul_const(const std::vector<CT>& in, const std::vector<double>& v,
                                   const std::vector<double>& target) {
  std::vector<LinItem> li;
  for (size_t i = 0; i < in.size(); ++i) {
    LinItem t{};
    t.a = in[i];
    t.va = v[i];
    t.target = target[i];
    li.push_back(t);
  }
  return lincomb(li, true);
}

// Plaintext operand of each item: its slot values (a dense prefix, or sparse
// (slot, value) pairs) encoded at 'scale', spread to the item's limbs and
// transformed.  product: x * pt, rescaled, scale := target (K of the encoding
// = target q_l / s, exact target scale); otherwise x + pt at x's scale.
std::vector<CT> Builder::plain_op(const std::vector<CT>& in, const std::vector<std::vector<double>>* dense,
                                  const std::vector<SparseSlots>* sparse, const std::vector<double>* target,
                                  bool product) {
  const int N = C.N;
  const uint32_t m2n = 2u * (uint32_t)N;
  const size_t mark = scratch_mark();
  std::vector<CT> out;
  std::vector<EncodeJob> j_enc;
  std::vector<IntSpreadJob> j_sp;
  std::vector<NttJob> j_ntt;
  std::vector<EwJob> j_op;
  // items with the same values, plaintext scale and level share one encoding
  std::map<std::tuple<int, double, std::vector<double>, std::vector<int>>, double*> done;
  for (size_t i = 0; i < in.size(); ++i) {
    const CT& x = in[i];
    const int nl = x.level + 1;
    double ps = x.scale;
    if (product) {
      const double ql = (double)C.mod[x.level];
      ps = (*target)[i] * ql;
      ps = ps / x.scale;
    }
    const auto key = sparse ? std::make_tuple(x.level, ps, (*sparse)[i].val, (*sparse)[i].slot)
                            : std::make_tuple(x.level, ps, (*dense)[i], std::vector<int>());
    double* pt = nullptr;
    auto hit = done.find(key);
    if (hit != done.end()) {
      pt = hit->second;
    } else {
      int64_t* m = (int64_t*)scratch(N);
      pt = scratch((size_t)nl * N);
      done.emplace(key, pt);
      EncodeJob ej{};
      if (sparse) {
        const SparseSlots& sp = (*sparse)[i];
        std::vector<uint32_t> g(sp.slot.size());
        for (size_t j = 0; j < sp.slot.size(); ++j) {
          // 5^slot mod 2N
          uint64_t r = 1, b = 5;
          for (uint32_t e = (uint32_t)sp.slot[j]; e; e >>= 1, b = b * b % m2n)
            if (e & 1) r = r * b % m2n;
          g[j] = (uint32_t)r;
        }
        ej.z = put(sp.val);
        ej.gs = put(g);
        ej.nnz = (int)sp.val.size();
      } else {
        ej.z = put((*dense)[i]);
        ej.nnz = (int)(*dense)[i].size();
      }
      ej.m = m;
      ej.scale_hi = ps * 2.0 / (double)N;
      ej.scale_lo = 0.0;
      j_enc.push_back(ej);
      j_sp.push_back(IntSpreadJob{m, pt, nl, nl});
      j_ntt.push_back(NttJob{pt, pt, nl, nl, 0, 0});
    }
    CT o = new_ct(x.level, x.scale);
    EwJob e{};
    e.o0 = c0(o); e.o1 = c1(o); e.a0 = c0(x); e.a1 = c1(x); e.b0 = pt;
    e.n_limbs = nl; e.n_chain = nl;
    e.op = product ? EW_PMUL : EW_PADD;
    j_op.push_back(e);
    out.push_back(o);
  }
  encode(j_enc);
  intspread(j_sp);
  ntt(j_ntt, false);
  ew(j_op);
  if (product) {
    rescale(out);
    if (err_code) return {};
    for (size_t i = 0; i < out.size(); ++i) out[i].scale = (*target)[i];
  }
  scratch_release(mark);
  return out;
}

// product with the encoded real vector z (slots 0..len-1), exact target scale
std::vector<CT> Builder::mul_plain(const std::vector<CT>& in, const std::vector<std::vector<double>>& z,
                                   const std::vector<double>& target) {
  return plain_op(in, &z, nullptr, &target, true);
}
std::vector<CT> Builder::mul_plain_sparse(const std::vector<CT>& in, const std::vector<SparseSlots>& z,
                                          const std::vector<double>& target) {
  return plain_op(in, nullptr, &z, &target, true);
}
std::vector<CT> Builder::add_plain_sparse(const std::vector<CT>& in, const std::vector<SparseSlots>& z) {
  return plain_op(in, nullptr, &z, nullptr, false);
}

// encryption of integer plaintexts (device int64 coefficient arrays) at the top level
void Builder::encrypt_into(const std::vector<const int64_t*>& m_dev, const std::vector<uint64_t>& seed, int purpose,
                           const std::vector<uint64_t>& sub, const double* sk, const std::vector<CT>& out) {
  const int N = C.N, L = C.n_q;
  const size_t mark = scratch_mark();
  std::vector<IntSpreadJob> j_sp;
  std::vector<SampleJob> j_s;
  std::vector<NttJob> j_ntt;
  std::vector<EwJob> j_enc;
  for (size_t i = 0; i < out.size(); ++i) {
    double* mm = scratch((size_t)L * N);
    double* e = scratch((size_t)L * N);
    const uint64_t tag = ((uint64_t)purpose << 56) | ((sub[i] & 0xFFFull) << 12);
    j_sp.push_back(IntSpreadJob{m_dev[i], mm, L, L});
    j_s.push_back(SampleJob{c1(out[i]), seed[i], tag, L, L, SAMPLE_UNIFORM, 0});
    j_s.push_back(SampleJob{e, seed[i], tag, L, L, SAMPLE_CBD, 0});
    j_ntt.push_back(NttJob{mm, mm, L, L, 0, 0});
    j_ntt.push_back(NttJob{e, e, L, L, 0, 0});
    j_ntt.push_back(NttJob{c1(out[i]), c1(out[i]), L, L, 0, 0});
    EwJob w{};
    w.o0 = c0(out[i]); w.a0 = mm; w.a1 = e; w.b0 = c1(out[i]); w.b1 = sk;
    w.n_limbs = L; w.n_chain = L; w.op = EW_ENC;
    j_enc.push_back(w);
  }
  intspread(j_sp);
  sample(j_s);
  ntt(j_ntt, false);
  ew(j_enc);
  scratch_release(mark);
}

// refresh stand-in: decrypt with the key owner's secret, lift m exactly from
// limbs 0 and 1, re-encrypt at the refresh level; scale kept
std::vector<CT> Builder::refresh(const std::vector<CT>& in, const std::vector<uint64_t>& seed,
                                 const std::vector<uint64_t>& index, const std::vector<int>* span) {
  if (C.boot_mode) {
    // items that read only slots [0, n) again take the sparse-slot bootstrap
    std::vector<size_t> sp, fu;
    for (size_t i = 0; i < in.size(); ++i) {
      const int w = span ? (*span)[i] : 0;
      (C.boot_sparse > 0 && w > 0 && w <= C.boot_sparse ? sp : fu).push_back(i);
    }
    std::vector<CT> out(in.size());
    for (int pass = 0; pass < 2; ++pass) {
      const std::vector<size_t>& idx = pass ? fu : sp;
      if (idx.empty()) continue;
      std::vector<CT> part;
      for (size_t i : idx) part.push_back(in[i]);
      // several such items: packed into shared full-slot bootstraps
      const bool pack = pass == 0 && C.boot_pack_min > 1 && idx.size() >= (size_t)C.boot_pack_min;
      std::vector<CT> o = pack ? bootstrap_packed(part) : bootstrap(part, pass == 0);
      if (err_code) return {};
      for (size_t k = 0; k < idx.size(); ++k) out[idx[k]] = o[k];
    }
    return out;
  }
  mark();
  const int N = C.N, L = C.refresh_level + 1;
  const double* rsk = refresh_sk ? refresh_sk : (dry ? C.T.mod : nullptr);
  if (!rsk) { fail(-3, "modulus chain exhausted: refreshing needs a key owner (or bootstrapping)"); return {}; }
  const size_t mark = scratch_mark();
  std::vector<CT> out;
  std::vector<EwJob> j_dec;
  std::vector<NttJob> j_inv, j_fwd, j_fwd2;
  std::vector<LiftJob> j_lift;
  std::vector<SampleJob> j_s;
  std::vector<EwJob> j_me, j_enc;
  for (size_t i = 0; i < in.size(); ++i) {
    const CT& x = in[i];
    if (x.level < 1) { fail(-3, "refresh needs two limbs"); return {}; }
    double* r = scratch(2 * (size_t)N);
    double* mm = scratch((size_t)L * N);
    double* e = scratch((size_t)L * N);
    EwJob d{};
    d.o0 = r; d.a0 = c0(x); d.a1 = c1(x); d.b0 = rsk;
    d.n_limbs = 2; d.n_chain = 2; d.op = EW_DEC2;
    j_dec.push_back(d);
    j_inv.push_back(NttJob{r, r, 2, 2, 0, 0});
    j_lift.push_back(LiftJob{r, r + N, mm, nullptr, L, 0});
    CT o = new_ct(L - 1, x.scale);
    const uint64_t tag = (5ull << 56) | ((index[i] & 0xFFFull) << 12);
    j_s.push_back(SampleJob{c1(o), seed[i], tag, L, L, SAMPLE_UNIFORM, 0});
    j_s.push_back(SampleJob{e, seed[i], tag, L, L, SAMPLE_CBD, 0});
    // m + e is formed in the coefficient domain, so one transform serves both
    EwJob me{};
    me.o0 = mm; me.a0 = mm; me.b0 = e;
    me.n_limbs = L; me.n_chain = L; me.op = EW_PADD;
    j_me.push_back(me);
    j_fwd.push_back(NttJob{mm, mm, L, L, 0, 0});
    j_fwd.push_back(NttJob{c1(o), c1(o), L, L, 0, 0});
    EwJob w{};
    w.o0 = c0(o); w.a1 = mm; w.b0 = c1(o); w.b1 = rsk;   // (m + e) - a s
    w.n_limbs = L; w.n_chain = L; w.op = EW_KEYB;
    j_enc.push_back(w);
    out.push_back(o);
  }
  ew(j_dec);
  ntt(j_inv, true);
  lift(j_lift);
  sample(j_s);
  ew(j_me);
  ntt(j_fwd, false);
  ew(j_enc);
  this->mark();
  counters[4] += (int64_t)in.size();
  scratch_release(mark);
  return out;
}

// odd degree-9 polynomial p(x) = (c1 x + c3 x^3) + x^4 (c5 x + c7 x^3) + x^8 (c9 x):
// baby steps x^2, x^3, x^4, giant step x^8 (three rounds of merged
// relinearise + rescale); B and C as constant combinations rescaled once, A
// unrescaled at the products' scale (formed inside the sum); x^4 B + x^8 C + A as one degree-2 sum,
// relinearised and rescaled once.  Depth 4, five relinearisations; output at
// level l-4 carrying (target q_{l-3}) / q_{l-3}.
std::vector<CT> Builder::eval_odd9(const std::vector<CT>& xs, const std::vector<const double*>& coef,
                                   const std::vector<double>& gain, const std::vector<double>& target) {
  const size_t n = xs.size();
  for (const CT& x : xs)
    if (x.level - 4 < C.min_level) { fail(-3, "eval_odd9: not enough levels"); return {}; }
  auto lower = [](CT x, int l) { x.level = l; x.slot = -1; return x; };
  std::vector<std::pair<CT, CT>> p;
  for (size_t i = 0; i < n; ++i) p.push_back({xs[i], xs[i]});
  std::vector<CT> x2 = mul_relin(p, true);
  if (err_code) return {};
  p.clear();
  for (size_t i = 0; i < n; ++i) p.push_back({x2[i], lower(xs[i], xs[i].level - 1)});
  for (size_t i = 0; i < n; ++i) p.push_back({x2[i], x2[i]});
  std::vector<CT> x34 = mul_relin(p, true);
  if (err_code) return {};
  std::vector<CT> x3(x34.begin(), x34.begin() + n), x4(x34.begin() + n, x34.end());
  p.clear();
  for (size_t i = 0; i < n; ++i) p.push_back({x4[i], x4[i]});
  std::vector<CT> x8 = mul_relin(p, true);
  if (err_code) return {};
  for (auto& v : x2) free_ct(v);
  std::vector<LinItem> bc, a;
  for (size_t i = 0; i < n; ++i) {
    const int l = xs[i].level;
    const double ta = target[i] * (double)C.mod[l - 3];
    const double g = gain[i];
    const double* c = coef[i];
    const CT xl2 = lower(xs[i], l - 2);
    LinItem B{};
    B.a = xl2; B.va = c[2] * g; B.b = x3[i]; B.vb = c[3] * g; B.has_b = true; B.target = ta / x4[i].scale;
    LinItem Cc{};
    Cc.a = xl2; Cc.va = c[4] * g; Cc.target = ta / x8[i].scale;
    bc.push_back(B);
    bc.push_back(Cc);
    LinItem A{};
    A.a = lower(xs[i], l - 3); A.va = c[0] * g; A.b = lower(x3[i], l - 3); A.vb = c[1] * g; A.has_b = true;
    A.target = ta;
    a.push_back(A);
  }
  std::vector<CT> kbc = lincomb(bc, true);
  if (err_code) return {};
  const size_t mark = scratch_mark();
  std::vector<TensorItem> ti;
  for (size_t i = 0; i < n; ++i) {
    TensorItem t{};
    t.a = lower(x4[i], xs[i].level - 3);
    t.b = kbc[2 * i];
    t.c = x8[i];
    t.e = kbc[2 * i + 1];
    t.has_ce = true;
    t.fl = a[i];   // A is formed inside the degree-2 sum
    t.has_fl = true;
    ti.push_back(t);
  }
  std::vector<Deg2> d = tensor2(ti);
  if (err_code) return {};
  for (auto& v : x3) free_ct(v);
  std::vector<CT> res = relin_rescale(d);
  if (err_code) return {};
  scratch_release(mark);
  for (size_t i = 0; i < n; ++i) {
    free_ct(kbc[2 * i]);
    free_ct(kbc[2 * i + 1]);
    free_ct(x4[i]);
    free_ct(x8[i]);
  }
  counters[5] += (int64_t)n;
  return res;
}

}  // namespace secpe

namespace secpe {

// ---------------------------------------------------------------------------
// bootstrapping (the paper refreshes by bootstrapping, Sec. 2.2 and Sec. 4.1):
// scale-down to level 0 at T_b = q_0 2^-ratio, ModRaise, CoeffToSlot,
// real/imaginary split by conjugation, EvalMod on both parts, recombination,
// SlotToCoeff.  The groups' plaintexts are built by secpe_boot_setup.
// ---------------------------------------------------------------------------

// level-0 ciphertexts: centred residues mod q_0 lifted to every chain prime;
// the result decrypts to t = m + q_0 I and is declared at scale q_0
std::vector<CT> Builder::mod_raise(const std::vector<CT>& in) {
  const int N = C.N, L = C.n_q;
  const size_t mark = scratch_mark();
  std::vector<CT> out;
  std::vector<NttJob> j_inv, j_fwd;
  std::vector<RaiseJob> j_r;
  for (const CT& x : in) {
    if (x.level != 0) { fail(-1, "mod_raise: input must be at level 0"); return {}; }
    CT o = new_ct(L - 1, (double)C.mod[0]);
    for (int w = 0; w < 2; ++w) {
      double* r = scratch(N);
      double* dst = w ? c1(o) : c0(o);
      j_inv.push_back(NttJob{w ? c1(x) : c0(x), r, 1, 1, 0, 0});
      j_r.push_back(RaiseJob{r, dst, L, 0});
      j_fwd.push_back(NttJob{dst, dst, L, L, 0, 0});
    }
    out.push_back(o);
  }
  ntt(j_inv, true);
  raise(j_r);
  ntt(j_fwd, false);
  scratch_release(mark);
  return out;
}

// slots times i (X^(N/2): 5^j = 1 mod 4) or -i (-X^(N/2)); exact, scale kept
std::vector<CT> Builder::mul_monomial_half(const std::vector<CT>& in, bool neg) {
  const double* mono = C.boot_mono ? C.boot_mono : (dry ? C.T.mod : nullptr);
  if (!mono) { fail(-1, "bootstrapping is not set up"); return {}; }
  std::vector<CT> out;
  std::vector<EwJob> j;
  for (const CT& x : in) {
    CT o = new_ct(x.level, x.scale);
    EwJob e{};
    e.o0 = c0(o); e.o1 = c1(o); e.a0 = c0(x); e.a1 = c1(x);
    e.b0 = mono + (neg ? (size_t)C.n_q * C.N : 0);
    e.n_limbs = x.level + 1; e.n_chain = x.level + 1;
    e.op = EW_PMUL;
    j.push_back(e);
    out.push_back(o);
  }
  ew(j);
  return out;
}

static int64_t fdiv(int64_t a, int64_t b) { return a >= 0 ? a / b : -((-a + b - 1) / b); }

// all groups of one direction; group g: out = sum_G RotL(sum_b pt_{G,b} * RotL(x, delta b), delta n1 G),
// rescaled once, scale := the group's output scale.  Inner sums are accumulated baby step by baby
// step, so one rotated copy of each input is alive at a time.
std::vector<CT> Builder::boot_transform(const std::vector<CT>& in, bool inverse, bool sparse) {
  const std::vector<BootGroup>& groups =
      sparse ? (inverse ? C.boot_cts_sp : C.boot_stc_sp) : (inverse ? C.boot_cts : C.boot_stc);
  if (groups.empty() || (!C.boot_ready && !dry)) { fail(-1, "bootstrapping is not set up"); return {}; }
  std::vector<CT> cur = in;
  bool own = false;
  for (const BootGroup& G : groups) {
    const size_t n = cur.size();
    if (G.e.empty() || G.e.size() != G.pt.size()) { fail(-1, "bootstrapping plaintexts are not set up"); return {}; }
    for (const CT& x : cur) {
      if (x.level != G.level) { fail(-1, "boot transform: input level does not match the set-up"); return {}; }
      if (x.scale != G.in_scale) { fail(-1, "boot transform: input scale does not match the set-up"); return {}; }
    }
    // giant steps present, in ascending order
    std::vector<int64_t> giants;
    for (int64_t e : G.e) giants.push_back(fdiv(e, G.n1));
    std::sort(giants.begin(), giants.end());
    giants.erase(std::unique(giants.begin(), giants.end()), giants.end());
    const size_t ng = giants.size();
    std::vector<CT> acc(n * ng);
    if (G.n1 <= 8 && ng <= 8) {
      // every baby step in use at once, then one fused launch for all inner sums
      std::vector<int> slot_of(G.n1, -1);
      std::vector<char> used(G.n1, 0);
      for (int64_t e : G.e) used[e - G.n1 * fdiv(e, G.n1)] = 1;
      std::vector<CT> rin;
      std::vector<int64_t> rst;
      for (int b = 1; b < G.n1; ++b) {
        if (!used[b]) continue;
        slot_of[b] = (int)(rin.size() / n);
        for (size_t it = 0; it < n; ++it) {
          rin.push_back(cur[it]);
          rst.push_back((int64_t)G.delta * b);
        }
      }
      // the baby steps share one ModUp per input (hoisted rotations)
      std::vector<CT> rb;
      if (!rin.empty()) {
        std::vector<int64_t> bst;
        for (size_t k = 0; k < rst.size(); k += n) bst.push_back(rst[k]);
        const size_t hm = scratch_mark();
        Hoisted hx = hoist(cur);
        rb = rotate_hoisted(hx, bst);
        scratch_release(hm);
        if (err_code) return {};
      }
      std::vector<BsgsJob> jb;
      for (size_t it = 0; it < n; ++it) {
        BsgsJob J{};
        J.n_limbs = G.level + 1;
        J.n_giants = (int)ng;
        J.n1 = G.n1;
        for (int b = 0; b < G.n1; ++b) {
          // an unused baby step has no plaintext; its input is only read
          const CT& xb = slot_of[b] < 0 ? cur[it] : rb[(size_t)slot_of[b] * n + it];
          J.x0[b] = c0(xb);
          J.x1[b] = c1(xb);
        }
        for (size_t gi = 0; gi < ng; ++gi) {
          acc[it * ng + gi] = new_ct(G.level, cur[it].scale * G.pscale);
          J.o0[gi] = c0(acc[it * ng + gi]);
          J.o1[gi] = c1(acc[it * ng + gi]);
        }
        for (size_t i = 0; i < G.e.size(); ++i) {
          const int64_t gg = fdiv(G.e[i], G.n1);
          const size_t gi = std::lower_bound(giants.begin(), giants.end(), gg) - giants.begin();
          J.pt[gi * 8 + (size_t)(G.e[i] - G.n1 * gg)] = G.pt[i];
        }
        jb.push_back(J);
      }
      bsgs(jb);
      for (CT& v : rb) free_ct(v);
    } else {
      std::vector<char> have(n * ng, 0);
      // the baby steps share one ModUp per input (hoisted rotations)
      bool any_baby = false;
      for (int64_t e : G.e) any_baby = any_baby || e != G.n1 * fdiv(e, G.n1);
      const size_t hm = scratch_mark();
      Hoisted hx;
      if (any_baby) hx = hoist(cur);
      for (int b = 0; b < G.n1; ++b) {
        std::vector<size_t> di;
        for (size_t i = 0; i < G.e.size(); ++i)
          if (G.e[i] - G.n1 * fdiv(G.e[i], G.n1) == b) di.push_back(i);
        if (di.empty()) continue;
        std::vector<CT> xb = cur;
        if (b > 0) {
          xb = rotate_hoisted(hx, {(int64_t)G.delta * b});
          if (err_code) return {};
        }
        // every accumulator gets at most one term per baby step: the first
        // term of an accumulator is a product, later ones accumulate
        std::vector<EwJob> j;
        for (size_t it = 0; it < n; ++it)
          for (size_t i : di) {
            const size_t gi = std::lower_bound(giants.begin(), giants.end(), fdiv(G.e[i], G.n1)) - giants.begin();
            const size_t a = it * ng + gi;
            EwJob e{};
            if (!have[a]) {
              acc[a] = new_ct(G.level, cur[it].scale * G.pscale);
              have[a] = 1;
              e.op = EW_PMUL;
            } else {
              e.c0 = c0(acc[a]); e.c1 = c1(acc[a]);
              e.op = EW_PMAC;
            }
            e.o0 = c0(acc[a]); e.o1 = c1(acc[a]);
            e.a0 = c0(xb[it]); e.a1 = c1(xb[it]);
            e.b0 = G.pt[i];
            e.n_limbs = G.level + 1; e.n_chain = G.level + 1;
            j.push_back(e);
          }
        ew(j);
        if (b > 0)
          for (CT& v : xb) free_ct(v);
      }
      scratch_release(hm);
    }
    // giant rotations, then the sum over giant steps
    std::vector<CT> rin;
    std::vector<int64_t> rst;
    std::vector<size_t> rpos;
    for (size_t it = 0; it < n; ++it)
      for (size_t gi = 0; gi < ng; ++gi)
        if (giants[gi] != 0) {
          rin.push_back(acc[it * ng + gi]);
          rst.push_back((int64_t)G.delta * G.n1 * giants[gi]);
          rpos.push_back(it * ng + gi);
        }
    if (!rin.empty()) {
      std::vector<CT> rout = rotate(rin, rst);
      if (err_code) return {};
      for (size_t k = 0; k < rpos.size(); ++k) {
        free_ct(acc[rpos[k]]);
        acc[rpos[k]] = rout[k];
      }
    }
    // the sum over giant steps, one launch per giant for every item at once
    std::vector<CT> nxt;
    if (ng == 1) {
      for (size_t it = 0; it < n; ++it) nxt.push_back(acc[it]);
    } else {
      std::vector<std::pair<CT, CT>> pr;
      for (size_t it = 0; it < n; ++it) pr.push_back({acc[it * ng], acc[it * ng + 1]});
      std::vector<CT> sum = add(pr, false);
      if (err_code) return {};
      for (size_t gi = 2; gi < ng; ++gi) {
        pr.clear();
        for (size_t it = 0; it < n; ++it) pr.push_back({sum[it], acc[it * ng + gi]});
        std::vector<CT> t = add(pr, false);
        if (err_code) return {};
        for (CT& v : sum) free_ct(v);
        sum = t;
      }
      for (size_t a = 0; a < n * ng; ++a) free_ct(acc[a]);
      nxt = sum;
    }
    const size_t mark = scratch_mark();
    rescale(nxt);
    scratch_release(mark);
    if (err_code) return {};
    for (CT& v : nxt) v.scale = G.out_scale;
    if (own)
      for (CT& v : cur) free_ct(v);
    cur = nxt;
    own = true;
  }
  return cur;
}

// relinearise degree-2 ciphertexts without rescaling: (d0, d1) + KS(d2)
std::vector<CT> Builder::relin(const std::vector<Deg2>& xs) {
  auto kit = C.keys.find(0);
  const double* rk = kit != C.keys.end() ? kit->second : (dry ? C.T.mod : nullptr);
  if (!rk) { fail(-4, "no relinearisation key"); return {}; }
  std::vector<CT> out;
  std::vector<KsItem> ks;
  for (const Deg2& x : xs) {
    if (x.sq0) { fail(-1, "relin: fused squares are not supported here"); return {}; }
    CT o = new_ct(x.level, x.scale);
    ks.push_back(KsItem{x.d2, x.level, rk, x.d0, x.d1, c0(o), c1(o), nullptr, nullptr, false});
    out.push_back(o);
  }
  key_switch(ks);
  counters[2] += (int64_t)xs.size();
  return out;
}

// x^2 relinearised, then rescaled by exact rounding (one level)
std::vector<CT> Builder::square_exact(const std::vector<CT>& xs) {
  std::vector<std::pair<CT, CT>> sq;
  for (const CT& x : xs) sq.push_back({x, x});
  std::vector<CT> p = mul_relin(sq, false);
  if (err_code) return {};
  const size_t mark = scratch_mark();
  rescale(p);
  scratch_release(mark);
  return p;
}

// EvalMod on u = x / (K+1) (Han-Ki 2020): p(u) = sum_j c_j T_j(u), the
// Chebyshev interpolant of cos(2 pi ((K+1) u - 1/4) / 2^r), then r double
// angles y <- 2 y^2 - 1.  p runs baby-step giant-step in the Chebyshev basis:
// baby steps T_1 .. T_(B-1) (B = 2^ceil(k/2), degree 2^k - 1), giant steps
// T_B .. T_(2^(k-1)); a node of degree < 2h splits by Chebyshev division into
// r + T_h q (q_0 = c_h, q_j = 2 c_(h+j), r_0 = c_0, r_j = c_j - c_(2h-j)),
// recursively down to combinations of the baby steps: one product per split,
// 11 products for degree 31, depth k + 1.  Every node lands exactly on the
// scale its parent needs; an r child made of baby steps is added, unrescaled,
// at the product's scale before relinearising and its constant after.  Basis
// products: T_2a = 2 T_a^2 - 1 (square, doubled, constant subtracted) and
// T_(a+b) = 2 T_a T_b - T_(a-b) ((2 T_a) (x) T_b plus -T_(a-b) at the
// product's scale).  Every product is relinearised and then rescaled by exact
// rounding: the merged relinearise-and-rescale rounds through an approximate
// conversion whose error (up to (alpha + 1) / 2 per coefficient) the double
// angles would amplify.

// T_j for every item by the product rules
void Builder::cheb_basis_step(std::vector<std::vector<CT>>& T, std::vector<std::vector<CT>>& T2, int j) {
  const size_t n = T[1].size();
  int a = 1;
  while (2 * a < j) a *= 2;
  const int b = j - a;
  const size_t mark = scratch_mark();
  if (b == a) {
    std::vector<CT> P = square_exact(T[a]);
    if (err_code) return;
    std::vector<LinItem> li;
    for (size_t i = 0; i < n; ++i) {
      LinItem t{};
      t.a = P[i];
      t.va = 2.0;
      t.target = P[i].scale;
      li.push_back(t);
    }
    std::vector<CT> P2 = lincomb(li, false);
    if (err_code) return;
    for (CT& v : P) free_ct(v);
    T[j] = add_const(P2, std::vector<double>(n, -1.0));
    if (err_code) return;
    for (CT& v : P2) free_ct(v);
  } else {
    if (T2[a].empty()) {
      std::vector<LinItem> li;
      for (size_t i = 0; i < n; ++i) {
        LinItem t{};
        t.a = T[a][i];
        t.va = 2.0;
        t.target = T[a][i].scale;
        li.push_back(t);
      }
      T2[a] = lincomb(li, false);
      if (err_code) return;
    }
    std::vector<LinItem> la;
    for (size_t i = 0; i < n; ++i) {
      LinItem t{};
      t.a = T[a - b][i];
      t.a.level = T2[a][i].level;
      t.a.slot = -1;
      t.va = -1.0;
      t.target = T2[a][i].scale * T[b][i].scale;
      la.push_back(t);
    }
    std::vector<CT> A = lincomb(la, false);
    if (err_code) return;
    std::vector<TensorItem> ti;
    for (size_t i = 0; i < n; ++i) {
      TensorItem t{};
      t.a = T2[a][i];
      t.b = T[b][i];
      t.f = A[i];
      t.has_f = true;
      ti.push_back(t);
    }
    std::vector<Deg2> d = tensor2(ti);
    if (err_code) return;
    T[j] = relin(d);
    if (err_code) return;
    rescale(T[j]);
    if (err_code) return;
    for (CT& v : A) free_ct(v);
  }
  scratch_release(mark);
}

// sum_{0 < j < nt} cf[j] T_j, every T_j lowered to level lv, at scale 'scale' (not rescaled)
std::vector<CT> Builder::cheb_combination(const std::vector<std::vector<CT>>& T, const double* cf, int nt, int lv,
                                          const std::vector<double>& scale) {
  const size_t n = T[1].size();
  std::vector<CT> acc;
  for (int j = 1; j < nt; ++j) {
    std::vector<LinItem> li;
    for (size_t i = 0; i < n; ++i) {
      LinItem t{};
      t.a = T[j][i];
      t.a.level = lv;
      t.a.slot = -1;
      t.va = cf[j];
      t.target = scale[i];
      if (!acc.empty()) { t.b = acc[i]; t.vb = 1.0; t.has_b = true; }
      li.push_back(t);
    }
    std::vector<CT> nx = lincomb(li, false);
    if (err_code) return {};
    for (CT& v : acc) free_ct(v);
    acc = nx;
  }
  return acc;
}

// sum_{j < 2^m} cf[j] T_j with scale exactly target[i]; baby steps below B at
// deepest level lb; a node of 2^m terms ends at level lb - 1 - (m - log2 B)
std::vector<CT> Builder::cheb_node(const std::vector<std::vector<CT>>& T, int B, int lb, const double* cf, int m,
                                   const std::vector<double>& target) {
  const size_t n = T[1].size();
  const int nt = 1 << m;
  if (nt <= B) {
    std::vector<double> pre(n);
    for (size_t i = 0; i < n; ++i) pre[i] = target[i] * (double)C.mod[lb];
    std::vector<CT> acc = cheb_combination(T, cf, nt, lb, pre);
    if (err_code) return {};
    const size_t mark = scratch_mark();
    rescale(acc);
    scratch_release(mark);
    if (err_code) return {};
    for (size_t i = 0; i < n; ++i) acc[i].scale = target[i];
    std::vector<CT> out = add_const(acc, std::vector<double>(n, cf[0]));
    if (err_code) return {};
    for (CT& v : acc) free_ct(v);
    return out;
  }
  const int h = nt / 2;
  std::vector<double> q(h), r(h);
  q[0] = cf[h];
  r[0] = cf[0];
  for (int j = 1; j < h; ++j) {
    q[j] = 2.0 * cf[h + j];
    r[j] = cf[j] - cf[2 * h - j];
  }
  int mb = 0;
  while ((1 << mb) < B) ++mb;
  const int lq = lb - 1 - (m - 1 - mb);
  std::vector<double> tq(n);
  for (size_t i = 0; i < n; ++i) {
    tq[i] = target[i] * (double)C.mod[lq];
    tq[i] = tq[i] / T[h][i].scale;
  }
  std::vector<CT> qc = cheb_node(T, B, lb, q.data(), m - 1, tq);
  if (err_code) return {};
  std::vector<double> sig(n);
  for (size_t i = 0; i < n; ++i) sig[i] = qc[i].scale * T[h][i].scale;
  std::vector<CT> A;
  if (h <= B) {
    A = cheb_combination(T, r.data(), h, lq, sig);
  } else {
    std::vector<CT> rc = cheb_node(T, B, lb, r.data(), m - 1, std::vector<double>(n, ldexp(1.0, C.log_scale)));
    if (err_code) return {};
    std::vector<LinItem> li;
    for (size_t i = 0; i < n; ++i) {
      LinItem t{};
      t.a = rc[i];
      t.va = 1.0;
      t.target = sig[i];
      li.push_back(t);
    }
    A = lincomb(li, false);
    for (CT& v : rc) free_ct(v);
  }
  if (err_code) return {};
  const size_t mark = scratch_mark();
  std::vector<TensorItem> ti;
  for (size_t i = 0; i < n; ++i) {
    TensorItem t{};
    t.a = qc[i];
    t.b = T[h][i];
    t.b.level = lq;
    t.b.slot = -1;
    t.f = A[i];
    t.has_f = true;
    ti.push_back(t);
  }
  std::vector<Deg2> d = tensor2(ti);
  if (err_code) return {};
  std::vector<CT> out = relin(d);
  if (err_code) return {};
  rescale(out);
  if (err_code) return {};
  scratch_release(mark);
  for (size_t i = 0; i < n; ++i) out[i].scale = target[i];
  for (CT& v : qc) free_ct(v);
  for (CT& v : A) free_ct(v);
  if (h <= B) {
    std::vector<CT> o2 = add_const(out, std::vector<double>(n, r[0]));
    if (err_code) return {};
    for (CT& v : out) free_ct(v);
    out = o2;
  }
  return out;
}

std::vector<CT> Builder::eval_mod(const std::vector<CT>& us) {
  const size_t n = us.size();
  const int deg = C.boot_deg;
  if (deg < 1 || (int)C.boot_cheb.size() != deg + 1) { fail(-1, "bootstrapping is not set up"); return {}; }
  const double delta = ldexp(1.0, C.log_scale);
  int k = 0;
  while ((1 << k) < deg + 1) ++k;
  for (const CT& u : us) {
    if (u.level != us[0].level) { fail(-1, "eval_mod: inputs must share the level"); return {}; }
    if (u.level - k - 1 - C.boot_r < 0) { fail(-3, "eval_mod: not enough levels"); return {}; }
  }
  int mb = (k + 1) / 2;
  if (mb < 1) mb = 1;
  const int B = 1 << mb;
  std::vector<std::vector<CT>> T(deg + 2), T2(deg + 2);
  T[1] = us;
  for (int j = 2; j < B; ++j) {
    cheb_basis_step(T, T2, j);
    if (err_code) return {};
  }
  for (int h = B; h < (1 << k); h *= 2) {
    cheb_basis_step(T, T2, h);
    if (err_code) return {};
  }
  const int lb = B > 2 ? T[B - 1][0].level : T[1][0].level;
  std::vector<CT> y = cheb_node(T, B, lb, C.boot_cheb.data(), k, std::vector<double>(n, delta));
  if (err_code) return {};
  for (int j = 2; j <= deg + 1; ++j)
    for (CT& v : T[j]) free_ct(v);
  for (int j = 1; j <= deg + 1; ++j)
    for (CT& v : T2[j]) free_ct(v);
  for (int i = 0; i < C.boot_r; ++i) {
    const size_t mark = scratch_mark();
    std::vector<CT> P = square_exact(y);
    if (err_code) return {};
    std::vector<LinItem> li;
    for (size_t t = 0; t < n; ++t) {
      LinItem it{};
      it.a = P[t];
      it.va = 2.0;
      it.target = P[t].scale;
      li.push_back(it);
    }
    std::vector<CT> P2 = lincomb(li, false);
    if (err_code) return {};
    for (CT& v : P) free_ct(v);
    std::vector<CT> y2 = add_const(P2, std::vector<double>(n, -1.0));
    if (err_code) return {};
    for (CT& v : P2) free_ct(v);
    for (CT& v : y) free_ct(v);
    y = y2;
    scratch_release(mark);
  }
  return y;
}

// the whole bootstrap of ciphertexts at level >= 1 with slot values |z| <= 1;
// results at boot_out_level with scale Delta.  Items run in chunks of
// boot_chunk so the temporaries of one chunk bound the workspace.
std::vector<CT> Builder::bootstrap(const std::vector<CT>& all, bool sparse) {
  if (C.boot_out_level < 0 || (!C.boot_ready && !dry)) { fail(-1, "bootstrapping is not set up"); return {}; }
  if (sparse && C.boot_sparse <= 0) { fail(-1, "sparse-slot bootstrapping is not set up"); return {}; }
  std::vector<CT> res;
  const size_t chunk = (size_t)std::max(1, C.boot_chunk);
  for (size_t c0 = 0; c0 < all.size(); c0 += chunk) {
    std::vector<CT> part(all.begin() + c0, all.begin() + std::min(all.size(), c0 + chunk));
    std::vector<CT> o = sparse ? bootstrap_sparse_chunk(part) : bootstrap_chunk(part);
    if (err_code) return {};
    res.insert(res.end(), o.begin(), o.end());
  }
  return res;
}

std::vector<CT> Builder::subsum(const std::vector<CT>& in, int n) {
  if (n < 1 || 2 * n > C.N / 2) { fail(-1, "subsum: n must satisfy 2n <= N/2"); return {}; }
  std::vector<CT> cur = in;
  bool own = false;
  for (int64_t r = n; r < C.N / 2; r *= 2) {
    std::vector<CT> rot = rotate(cur, std::vector<int64_t>(cur.size(), r));
    if (err_code) return {};
    std::vector<std::pair<CT, CT>> pr;
    for (size_t i = 0; i < cur.size(); ++i) pr.push_back({cur[i], rot[i]});
    std::vector<CT> nx = add(pr, false);
    if (err_code) return {};
    for (CT& v : rot) free_ct(v);
    if (own)
      for (CT& v : cur) free_ct(v);
    cur = nx;
    own = true;
  }
  return cur;
}

// Sparse-slot bootstrap of n = boot_sparse slots: the mask of slots [0, n)
// replaces the scale-down constant; the trace at level 0 makes the message
// n-periodic; ModRaise; the trace again; the n-slot CoeffToSlot, whose last
// group writes [w, 0] with period 2n; [re, 0] = w + conj(w) and [im, 0] =
// -i (w - conj(w)) join as [re, im] = [re, 0] + RotR([im, 0], n); one EvalMod;
// the n-slot SlotToCoeff of re + i im.  Same depth as the full pipeline.
std::vector<CT> Builder::bootstrap_sparse_chunk(const std::vector<CT>& in) {
  const size_t n = in.size();
  const int ns = C.boot_sparse, S = C.N / 2;
  const double tb = ldexp((double)C.mod[0], -C.boot_ratio);
  std::vector<CT> x1;
  std::vector<std::vector<double>> mask;
  std::vector<double> tg;
  for (const CT& x : in) {
    if (x.level < 1) { fail(-3, "bootstrap: input needs level >= 1"); return {}; }
    CT v = x;
    v.level = 1;
    v.slot = -1;
    x1.push_back(v);
    mask.push_back(std::vector<double>(ns, 1.0));
    tg.push_back(tb);
  }
  std::vector<CT> x0 = mul_plain(x1, mask, tg);
  if (err_code) return {};
  std::vector<CT> t0 = subsum(x0, ns);
  if (err_code) return {};
  for (CT& v : x0) free_ct(v);
  std::vector<CT> r = mod_raise(t0);
  if (err_code) return {};
  for (CT& v : t0) free_ct(v);
  std::vector<CT> rt = subsum(r, ns);
  if (err_code) return {};
  for (CT& v : r) free_ct(v);
  std::vector<CT> y = boot_transform(rt, true, true);
  if (err_code) return {};
  for (CT& v : rt) free_ct(v);
  std::vector<CT> yc = rotate(y, std::vector<int64_t>(n, kConjStep));
  if (err_code) return {};
  std::vector<std::pair<CT, CT>> pr;
  for (size_t i = 0; i < n; ++i) pr.push_back({y[i], yc[i]});
  std::vector<CT> re, df;
  add_sub(pr, df, re);
  if (err_code) return {};
  for (CT& v : y) free_ct(v);
  for (CT& v : yc) free_ct(v);
  std::vector<CT> im = mul_monomial_half(df, true);
  if (err_code) return {};
  for (CT& v : df) free_ct(v);
  std::vector<CT> imr = rotate(im, std::vector<int64_t>(n, (int64_t)S - ns));
  if (err_code) return {};
  for (CT& v : im) free_ct(v);
  pr.clear();
  for (size_t i = 0; i < n; ++i) pr.push_back({re[i], imr[i]});
  std::vector<CT> u = add(pr, false);
  if (err_code) return {};
  for (CT& v : re) free_ct(v);
  for (CT& v : imr) free_ct(v);
  std::vector<CT> e = eval_mod(u);
  if (err_code) return {};
  for (CT& v : u) free_ct(v);
  std::vector<CT> out = boot_transform(e, false, true);
  if (err_code) return {};
  for (CT& v : e) free_ct(v);
  for (const CT& v : out)
    if (v.level != C.boot_out_level) { fail(-1, "bootstrap: level plan mismatch"); return {}; }
  counters[4] += (int64_t)n;
  return out;
}

std::vector<CT> Builder::bootstrap_chunk(const std::vector<CT>& in) {
  const size_t n = in.size();
  const double tb = ldexp((double)C.mod[0], -C.boot_ratio);
  std::vector<LinItem> li;
  for (const CT& x : in) {
    if (x.level < 1) { fail(-3, "bootstrap: input needs level >= 1"); return {}; }
    LinItem t{};
    t.a = x;
    t.a.level = 1;
    t.a.slot = -1;
    t.va = 1.0;
    t.target = tb;
    li.push_back(t);
  }
  std::vector<CT> x0 = lincomb(li, true);
  if (err_code) return {};
  std::vector<CT> out = boot_core_full(x0);
  if (err_code) return {};
  counters[4] += (int64_t)n;
  return out;
}

std::vector<CT> Builder::boot_core_full(std::vector<CT> x0) {
  const size_t n = x0.size();
  std::vector<CT> r = mod_raise(x0);
  if (err_code) return {};
  for (CT& v : x0) free_ct(v);
  std::vector<CT> y = boot_transform(r, true);
  if (err_code) return {};
  for (CT& v : r) free_ct(v);
  std::vector<CT> yc = rotate(y, std::vector<int64_t>(n, kConjStep));
  if (err_code) return {};
  std::vector<std::pair<CT, CT>> pr;
  for (size_t i = 0; i < n; ++i) pr.push_back({y[i], yc[i]});
  std::vector<CT> re = add(pr, false);
  std::vector<CT> df = add(pr, true);
  if (err_code) return {};
  for (CT& v : y) free_ct(v);
  for (CT& v : yc) free_ct(v);
  std::vector<CT> im = mul_monomial_half(df, true);
  if (err_code) return {};
  for (CT& v : df) free_ct(v);
  std::vector<CT> both = re;
  both.insert(both.end(), im.begin(), im.end());
  std::vector<CT> e = eval_mod(both);
  if (err_code) return {};
  for (CT& v : both) free_ct(v);
  std::vector<CT> ei(e.begin() + n, e.end());
  std::vector<CT> imi = mul_monomial_half(ei, false);
  if (err_code) return {};
  pr.clear();
  for (size_t i = 0; i < n; ++i) pr.push_back({e[i], imi[i]});
  std::vector<CT> w = add(pr, false);
  if (err_code) return {};
  for (CT& v : e) free_ct(v);
  for (CT& v : imi) free_ct(v);
  std::vector<CT> out = boot_transform(w, false);
  if (err_code) return {};
  for (CT& v : w) free_ct(v);
  for (const CT& v : out)
    if (v.level != C.boot_out_level) { fail(-1, "bootstrap: level plan mismatch"); return {}; }
  return out;
}

// Window-packed bootstrap: ciphertexts that are read only on slots [0, W)
// again (W = boot_sparse) share full-slot bootstraps, N/2W per bootstrap, in
// groups of m taken in order.  Per group:
//   scale-down  the sparse-slot mask of [0, W) at q_0 / 2^ratio, to level 0;
//   pack        T = sum_i RotL(z_i, i W), z_i = v_(m-1-i): at round b node t
//               becomes node 2t + RotL(node 2t+1, 2^b W) (an odd last node
//               passes through); P = RotL(T, ((N/2W - m + 1) mod N/2W) W), one
//               rotation by 2^b W per set bit, lowest first; P holds input
//               j's window at slots [jW, jW + W), zeros elsewhere;
//   bootstrap   the full pipeline from ModRaise on;
//   unpack      U_0 = P'; at round b each U_o, o < 2^b, gives
//               U_(o + 2^b) = RotL(U_o, 2^b W) while o + 2^b < m.
// Every rotation is by a power-of-two multiple of W below N/2: the keys of
// the sparse-slot trace.  A round's rotations share one key, so each round
// is one batched key switch over every group.
std::vector<CT> Builder::bootstrap_packed(const std::vector<CT>& in) {
  if (C.boot_out_level < 0 || (!C.boot_ready && !dry)) { fail(-1, "bootstrapping is not set up"); return {}; }
  const int W = C.boot_sparse, S = C.N / 2;
  if (W <= 0) { fail(-1, "packed bootstrapping needs the sparse-slot width"); return {}; }
  const int per = S / W;
  const size_t k = in.size();
  const double tb = ldexp((double)C.mod[0], -C.boot_ratio);
  std::vector<CT> x1;
  std::vector<std::vector<double>> mask;
  std::vector<double> tg;
  for (const CT& x : in) {
    if (x.level < 1) { fail(-3, "bootstrap: input needs level >= 1"); return {}; }
    CT v = x;
    v.level = 1;
    v.slot = -1;
    x1.push_back(v);
    mask.push_back(std::vector<double>(W, 1.0));
    tg.push_back(tb);
  }
  std::vector<CT> v = mul_plain(x1, mask, tg);
  if (err_code) return {};
  std::vector<std::vector<CT>> z;
  std::vector<int> gm;
  for (size_t p0 = 0; p0 < k; p0 += per) {
    const int m = (int)std::min<size_t>(per, k - p0);
    std::vector<CT> zz;
    for (int i = 0; i < m; ++i) zz.push_back(v[p0 + m - 1 - i]);
    z.push_back(zz);
    gm.push_back(m);
  }
  const size_t ng = z.size();
  for (int b = 0;; ++b) {
    std::vector<CT> rin;
    for (size_t g = 0; g < ng; ++g)
      for (size_t t = 0; 2 * t + 1 < z[g].size(); ++t) rin.push_back(z[g][2 * t + 1]);
    if (rin.empty()) break;
    std::vector<CT> r = rotate(rin, std::vector<int64_t>(rin.size(), (int64_t)W << b));
    if (err_code) return {};
    std::vector<std::pair<CT, CT>> pr;
    size_t q = 0;
    for (size_t g = 0; g < ng; ++g)
      for (size_t t = 0; 2 * t + 1 < z[g].size(); ++t) pr.push_back({z[g][2 * t], r[q++]});
    std::vector<CT> sum = add(pr, false);
    if (err_code) return {};
    for (CT& c : r) free_ct(c);
    q = 0;
    for (size_t g = 0; g < ng; ++g) {
      std::vector<CT> nz;
      for (size_t t = 0; 2 * t < z[g].size(); ++t) {
        if (2 * t + 1 < z[g].size()) {
          free_ct(z[g][2 * t]);
          free_ct(z[g][2 * t + 1]);
          nz.push_back(sum[q++]);
        } else {
          nz.push_back(z[g][2 * t]);
        }
      }
      z[g] = nz;
    }
  }
  std::vector<CT> P;
  for (size_t g = 0; g < ng; ++g) P.push_back(z[g][0]);
  for (int b = 0; (1 << b) < per; ++b) {
    std::vector<CT> rin;
    std::vector<size_t> who;
    for (size_t g = 0; g < ng; ++g)
      if (((per - gm[g] + 1) % per) & (1 << b)) {
        rin.push_back(P[g]);
        who.push_back(g);
      }
    if (rin.empty()) continue;
    std::vector<CT> r = rotate(rin, std::vector<int64_t>(rin.size(), (int64_t)W << b));
    if (err_code) return {};
    for (size_t i = 0; i < who.size(); ++i) {
      free_ct(P[who[i]]);
      P[who[i]] = r[i];
    }
  }
  std::vector<CT> Pb;
  const size_t chunk = (size_t)std::max(1, C.boot_chunk);
  for (size_t c0 = 0; c0 < ng; c0 += chunk) {
    std::vector<CT> part(P.begin() + c0, P.begin() + std::min(ng, c0 + chunk));
    std::vector<CT> o = boot_core_full(part);
    if (err_code) return {};
    Pb.insert(Pb.end(), o.begin(), o.end());
  }
  std::vector<std::vector<CT>> U(ng);
  for (size_t g = 0; g < ng; ++g) {
    U[g].resize(gm[g]);
    U[g][0] = Pb[g];
  }
  for (int b = 0; (1 << b) < per; ++b) {
    std::vector<CT> rin;
    std::vector<std::pair<size_t, int>> who;
    for (size_t g = 0; g < ng; ++g)
      for (int o = 0; o < (1 << b) && o + (1 << b) < gm[g]; ++o) {
        rin.push_back(U[g][o]);
        who.push_back({g, o + (1 << b)});
      }
    if (rin.empty()) break;
    std::vector<CT> r = rotate(rin, std::vector<int64_t>(rin.size(), (int64_t)W << b));
    if (err_code) return {};
    for (size_t i = 0; i < who.size(); ++i) U[who[i].first][who[i].second] = r[i];
  }
  std::vector<CT> out;
  for (size_t g = 0; g < ng; ++g) out.insert(out.end(), U[g].begin(), U[g].end());
  counters[4] += (int64_t)k;
  return out;
}

}  // namespace secpe
