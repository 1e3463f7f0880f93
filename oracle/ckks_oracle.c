/*
 * ckks_oracle.c -- plain, slow CPU reference of RNS-CKKS and of the SecPE
 * encrypted Argmax.
 *
 * TEST INFRASTRUCTURE ONLY.  Only tests/, the smoke check and the CPU-baseline
 * leg of the benchmark may load this library.  It shares no code, headers or
 * tables with the GPU library; the only things both sides agree on are the
 * conventions written out below (each side implements them on its own).
 *
 * Paper: "SecPE: Secure Prompt Ensembling for Private and Robust Large Language
 * Models" (arXiv 2502.00847).
 *   - RNS-CKKS over R_Q = Z_Q[X]/(X^N+1), Q = prod q_i            (Sec. 2.2)
 *   - homomorphic add/sub/mult, RotL/RotR                          (Sec. 2.2)
 *   - Argmax z_i = Sign(y_i - y_max) + 1                           (Sec. 3.2, Eq. 2)
 *   - Sign = f^{d_f}(g^{d_g}(x)), degree-9 f and g, BSGS evaluation (Sec. 3.2, Eq. 3-4)
 *   - normalisation (x - D_min)/(D_max - D_min)                    (Sec. 3.2, Eq. 5)
 *   - Max(a,b) = (a+b)/2 + (a-b)/2 * Sign(a-b)                     (Sec. 3.2, Eq. 6)
 *   - ARGMAX / QuickMax                                            (Sec. 3.2, Algorithm 1)
 *   - bootstrapping refreshes a low-level ciphertext               (Sec. 2.2; Sec. 4.1)
 *
 * Arithmetic is deliberately the most obvious kind: every modular product is a
 * 128-bit product reduced with '%', every NTT is the textbook bit-reversed
 * radix-2 transform of a psi-twisted vector, basis conversion and rescaling are
 * the formulas themselves.  Ciphertexts are held in the coefficient domain with
 * canonical residues in [0, q).
 *
 * Conventions the paper leaves open (each fixed here and in the GPU library
 * independently):
 *   primes   chain: primes = 1 mod 2N nearest 2^qbits, alternately the next one
 *            below and the next one above (q0 below); special: the largest
 *            primes = 1 mod 2N below 2^pbits.
 *   PRNG     SplitMix64 (Steele, Lea, Flood 2014) used counter-based:
 *            key = mix(seed ^ mix(tag)), draw(key,i) = mix(key + (i+1)*gamma).
 *   samplers ternary secret mulhi64(r,3)-1; error = centred binomial eta=21;
 *            uniform mod q = floor(((r0<<64)|r1) * q / 2^128).
 *   encode   m_k = round-half-away(scale * 2/N * sum_j z_j cos(pi*(5^j k mod 2N)/N)),
 *            evaluated in binary128.
 *   rescale  c' = (c - [c]_{q_l}centred) * q_l^{-1}.
 *   keyswitch hybrid: digits of alpha consecutive chain primes, gadget
 *            P*(Q/D_j)*[(Q/D_j)^{-1}]_{D_j}; ModUp = approximate conversion
 *            sum_i [x_i (D/q_i)^{-1}]_{q_i} (D/q_i); ModDown = (c - Conv_P(c)) * P^{-1}.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <stdio.h>
#include <math.h>
#include <quadmath.h>

typedef unsigned __int128 u128;
typedef __int128 i128;

#define ORC_API __attribute__((visibility("default")))

static void die(const char* msg) {
  fprintf(stderr, "ckks_oracle: %s\n", msg);
  abort();
}

/* ------------------------------------------------------------------------- */
/* modular arithmetic                                                         */
/* ------------------------------------------------------------------------- */
static inline uint64_t mmul(uint64_t a, uint64_t b, uint64_t q) { return (uint64_t)(((u128)a * b) % q); }
static inline uint64_t madd(uint64_t a, uint64_t b, uint64_t q) { return (uint64_t)(((u128)a + b) % q); }
static inline uint64_t msub(uint64_t a, uint64_t b, uint64_t q) { return (uint64_t)(((u128)a + q - b) % q); }
static inline uint64_t mneg(uint64_t a, uint64_t q) { return a == 0 ? 0 : q - a; }
static uint64_t mpow(uint64_t a, uint64_t e, uint64_t q) {
  uint64_t r = 1 % q;
  a %= q;
  while (e) {
    if (e & 1) r = mmul(r, a, q);
    a = mmul(a, a, q);
    e >>= 1;
  }
  return r;
}
static uint64_t minv(uint64_t a, uint64_t q) { return mpow(a, q - 2, q); } /* q prime */
static uint64_t from_i128(i128 x, uint64_t q) {
  i128 r = x % (i128)q;
  if (r < 0) r += q;
  return (uint64_t)r;
}

static int is_prime(uint64_t n) {
  static const uint64_t bases[12] = {2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37};
  if (n < 2) return 0;
  for (int i = 0; i < 12; ++i) {
    if (n % bases[i] == 0) return n == bases[i];
  }
  uint64_t d = n - 1;
  int s = 0;
  while ((d & 1) == 0) { d >>= 1; ++s; }
  for (int i = 0; i < 12; ++i) {
    uint64_t x = mpow(bases[i], d, n);
    if (x == 1 || x == n - 1) continue;
    int composite = 1;
    for (int r = 1; r < s; ++r) {
      x = mmul(x, x, n);
      if (x == n - 1) { composite = 0; break; }
    }
    if (composite) return 0;
  }
  return 1;
}

/* ------------------------------------------------------------------------- */
/* counter-based SplitMix64                                                   */
/* ------------------------------------------------------------------------- */
#define SM_GAMMA 0x9E3779B97F4A7C15ULL
static inline uint64_t sm_mix(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}
static inline uint64_t sm_key(uint64_t seed, uint64_t tag) { return sm_mix(seed ^ sm_mix(tag)); }
static inline uint64_t sm_draw(uint64_t key, uint64_t i) { return sm_mix(key + (i + 1) * SM_GAMMA); }

enum { PUR_SECRET = 1, PUR_RELIN = 2, PUR_GALOIS = 3, PUR_ENCRYPT = 4, PUR_REFRESH = 5 };
#define LIMB_NONE 0xFFFu
static inline uint64_t make_tag(uint64_t purpose, uint64_t obj, uint64_t sub, uint64_t limb) {
  return (purpose << 56) | ((obj & 0xFFFFFFFFull) << 24) | ((sub & 0xFFFull) << 12) | (limb & 0xFFFull);
}

static int64_t sample_ternary(uint64_t key, uint64_t i) {
  uint64_t r = sm_draw(key, i);
  return (int64_t)(uint64_t)(((u128)r * 3) >> 64) - 1;
}
/* sparse ternary: nonzero iff the top log2 N bits of the draw are below h
   (probability h/N), sign from the lowest bit */
static int64_t sample_sparse(uint64_t key, uint64_t i, int log_n, int h) {
  uint64_t r = sm_draw(key, i);
  if ((r >> (64 - log_n)) >= (uint64_t)h) return 0;
  return (r & 1) ? -1 : 1;
}
static int64_t sample_cbd21(uint64_t key, uint64_t i) {
  uint64_t r = sm_draw(key, i);
  const uint64_t m = (1ull << 21) - 1;
  return (int64_t)__builtin_popcountll(r & m) - (int64_t)__builtin_popcountll((r >> 21) & m);
}
static uint64_t sample_uniform(uint64_t key, uint64_t i, uint64_t q) {
  uint64_t hi = sm_draw(key, 2 * i), lo = sm_draw(key, 2 * i + 1);
  u128 t = (u128)hi * q + (((u128)lo * q) >> 64);
  return (uint64_t)(t >> 64);
}

/* ------------------------------------------------------------------------- */
/* context                                                                    */
/* ------------------------------------------------------------------------- */
/* the encoded plaintexts of one linear-transform group at one plaintext scale */
struct boot_pt {
  int inverse, g, ns;   /* ns: slots of the transform (N/2, or the sparse n) */
  double pscale;
  int64_t** m;          /* [slot offset] encoded (pre-rotated) diagonal, or NULL */
  struct boot_pt* next;
};

typedef struct {
  uint64_t g;           /* Galois element; 0 marks the relinearisation key */
  uint64_t*** b;        /* [digit][limb] NTT-domain vectors, limb over all primes */
  uint64_t*** a;
} orc_key;

typedef struct {
  int log_n, n;
  int n_q, n_p, alpha, dnum;
  int log_scale;
  int dg, df;
  int min_level;
  int refresh_level;    /* level a refreshed ciphertext is re-encrypted at */
  int refresh_level_set; /* the level the parameters asked for */
  int secret_h;         /* > 0: sparse secret, each coefficient nonzero w.p. h/N */
  int boot_mode;        /* 1: refreshes are bootstraps */
  int textbook;         /* 1: every product relinearised, then rescaled (no merged op) */
  int boot_K, boot_r, boot_deg, boot_ratio, boot_groups;
  int boot_out_level;   /* level of a bootstrapped ciphertext (-1: not set up) */
  int boot_sparse;      /* n > 0: slots [0, n) kept by the sparse-slot bootstrap */
  double* boot_cheb;    /* Chebyshev coefficients c_0..c_deg of the scaled cosine */
  struct boot_pt* boot_cache; /* encoded diagonals, by (direction, group, scale) */
  uint64_t* mod;        /* n_q chain primes, then n_p special primes */
  /* per prime NTT tables */
  uint64_t** psi_pow;   /* psi^i */
  uint64_t** psi_ipow;  /* psi^-i */
  uint64_t** om_pow;    /* omega^i, omega = psi^2 */
  uint64_t** om_ipow;   /* omega^-i */
  uint64_t* n_inv;
  __float128* cos_tab;  /* cos(pi t / N), t < 2N */
  uint64_t* rot_group;  /* 5^j mod 2N, j < N/2 */
  int64_t* s;           /* secret key, ternary */
  orc_key* keys;
  int n_keys;
  int64_t counters[8];
} orc_ctx;

enum { CNT_SIGN = 0, CNT_ROT = 1, CNT_RELIN = 2, CNT_KS = 3, CNT_REFRESH = 4, CNT_POLY = 5, CNT_MAX = 6 };

static void* xcalloc(size_t n, size_t sz) {
  void* p = calloc(n, sz);
  if (!p && n && sz) die("out of memory");
  return p;
}

/* first prime = 1 mod 2N strictly below 'below', stepping down by 2N */
static uint64_t prime_below(uint64_t start /* = 1 mod 2N */, uint64_t m2n, const uint64_t* taken, int n_taken) {
  for (uint64_t c = start; c > m2n; c -= m2n) {
    if (!is_prime(c)) continue;
    int dup = 0;
    for (int i = 0; i < n_taken; ++i) dup |= taken[i] == c;
    if (!dup) return c;
  }
  die("no prime found");
  return 0;
}

static void make_primes(orc_ctx* c, int q_bits, int p_bits) {
  uint64_t m2n = 2ull * (uint64_t)c->n;
  uint64_t base = 1ull << q_bits;
  uint64_t below = base + 1 - m2n; /* next candidate below 2^qbits */
  uint64_t above = base + 1;        /* next candidate above 2^qbits */
  int k = 0;
  while (k < c->n_q) {
    if ((k & 1) == 0) {
      while (!is_prime(below)) below -= m2n;
      c->mod[k++] = below;
      below -= m2n;
    } else {
      while (!is_prime(above)) above += m2n;
      c->mod[k++] = above;
      above += m2n;
    }
  }
  uint64_t top = (1ull << p_bits) + 1 - m2n;
  for (int j = 0; j < c->n_p; ++j) {
    uint64_t p = prime_below(top, m2n, c->mod, c->n_q + j);
    c->mod[c->n_q + j] = p;
    top = p - m2n;
  }
}

/* smallest quadratic non-residue x, psi = x^((q-1)/2N) has order exactly 2N */
static uint64_t find_psi(uint64_t q, uint64_t n) {
  for (uint64_t x = 2;; ++x) {
    if (mpow(x, (q - 1) / 2, q) == q - 1) return mpow(x, (q - 1) / (2 * n), q);
  }
}

/* refresh_level: level of a refreshed ciphertext (<= 0 or above the top: the top level) */
ORC_API void* orc_create(int log_n, int n_q, int q_bits, int n_p, int p_bits, int log_scale,
                         int dg, int df, int min_level, int refresh_level) {
  if (log_n < 3 || log_n > 17 || n_q < 2 || n_p < 1 || q_bits > 61 || p_bits > 61) die("bad parameters");
  orc_ctx* c = (orc_ctx*)xcalloc(1, sizeof(orc_ctx));
  c->log_n = log_n;
  c->n = 1 << log_n;
  c->n_q = n_q;
  c->n_p = n_p;
  c->alpha = n_p;
  c->dnum = (n_q + n_p - 1) / n_p;
  c->log_scale = log_scale;
  c->dg = dg;
  c->df = df;
  c->min_level = min_level;
  c->refresh_level = (refresh_level <= 0 || refresh_level > n_q - 1) ? n_q - 1 : refresh_level;
  c->boot_out_level = -1;
  c->refresh_level_set = c->refresh_level;
  int np = n_q + n_p, n = c->n;
  c->mod = (uint64_t*)xcalloc(np, sizeof(uint64_t));
  make_primes(c, q_bits, p_bits);
  c->psi_pow = (uint64_t**)xcalloc(np, sizeof(uint64_t*));
  c->psi_ipow = (uint64_t**)xcalloc(np, sizeof(uint64_t*));
  c->om_pow = (uint64_t**)xcalloc(np, sizeof(uint64_t*));
  c->om_ipow = (uint64_t**)xcalloc(np, sizeof(uint64_t*));
  c->n_inv = (uint64_t*)xcalloc(np, sizeof(uint64_t));
  for (int t = 0; t < np; ++t) {
    uint64_t q = c->mod[t];
    uint64_t psi = find_psi(q, (uint64_t)n), psi_i = minv(psi, q);
    uint64_t om = mmul(psi, psi, q), om_i = mmul(psi_i, psi_i, q);
    c->psi_pow[t] = (uint64_t*)xcalloc(n, 8);
    c->psi_ipow[t] = (uint64_t*)xcalloc(n, 8);
    c->om_pow[t] = (uint64_t*)xcalloc(n, 8);
    c->om_ipow[t] = (uint64_t*)xcalloc(n, 8);
    uint64_t a = 1, b = 1, d = 1, e = 1;
    for (int i = 0; i < n; ++i) {
      c->psi_pow[t][i] = a; a = mmul(a, psi, q);
      c->psi_ipow[t][i] = b; b = mmul(b, psi_i, q);
      c->om_pow[t][i] = d; d = mmul(d, om, q);
      c->om_ipow[t][i] = e; e = mmul(e, om_i, q);
    }
    c->n_inv[t] = minv((uint64_t)n, q);
  }
  c->cos_tab = (__float128*)xcalloc(2 * (size_t)n, sizeof(__float128));
  for (int t = 0; t < 2 * n; ++t) c->cos_tab[t] = cosq(M_PIq * (__float128)t / (__float128)n);
  c->rot_group = (uint64_t*)xcalloc(n / 2, 8);
  uint64_t g = 1;
  for (int j = 0; j < n / 2; ++j) { c->rot_group[j] = g; g = (g * 5) % (2 * (uint64_t)n); }
  return c;
}

static void free_key(orc_ctx* c, orc_key* k) {
  for (int j = 0; j < c->dnum; ++j) {
    for (int t = 0; t < c->n_q + c->n_p; ++t) { free(k->b[j][t]); free(k->a[j][t]); }
    free(k->b[j]); free(k->a[j]);
  }
  free(k->b); free(k->a);
}

ORC_API void orc_destroy(void* h) {
  orc_ctx* c = (orc_ctx*)h;
  if (!c) return;
  int np = c->n_q + c->n_p;
  for (int t = 0; t < np; ++t) { free(c->psi_pow[t]); free(c->psi_ipow[t]); free(c->om_pow[t]); free(c->om_ipow[t]); }
  free(c->psi_pow); free(c->psi_ipow); free(c->om_pow); free(c->om_ipow); free(c->n_inv);
  free(c->cos_tab); free(c->rot_group); free(c->s); free(c->boot_cheb);
  for (struct boot_pt* e = c->boot_cache; e;) {
    struct boot_pt* nx = e->next;
    for (int d = 0; d < c->n / 2; ++d) free(e->m[d]);
    free(e->m);
    free(e);
    e = nx;
  }
  for (int i = 0; i < c->n_keys; ++i) free_key(c, &c->keys[i]);
  free(c->keys); free(c->mod); free(c);
}

ORC_API int orc_num_primes(void* h) { orc_ctx* c = (orc_ctx*)h; return c->n_q + c->n_p; }
ORC_API void orc_primes(void* h, uint64_t* out) {
  orc_ctx* c = (orc_ctx*)h;
  memcpy(out, c->mod, sizeof(uint64_t) * (size_t)(c->n_q + c->n_p));
}
ORC_API void orc_counters(void* h, int64_t* out) { memcpy(out, ((orc_ctx*)h)->counters, sizeof(int64_t) * 8); }
ORC_API void orc_reset_counters(void* h) { memset(((orc_ctx*)h)->counters, 0, sizeof(int64_t) * 8); }

/* ------------------------------------------------------------------------- */
/* negacyclic NTT: twist by psi^i, textbook cyclic radix-2 transform          */
/* ------------------------------------------------------------------------- */
static void bit_reverse(uint64_t* a, int n) {
  for (int i = 1, j = 0; i < n; ++i) {
    int bit = n >> 1;
    for (; j & bit; bit >>= 1) j ^= bit;
    j ^= bit;
    if (i < j) { uint64_t t = a[i]; a[i] = a[j]; a[j] = t; }
  }
}
static void cyclic_ntt(uint64_t* a, int n, const uint64_t* wpow, uint64_t q) {
  bit_reverse(a, n);
  for (int len = 2; len <= n; len <<= 1) {
    int half = len >> 1, step = n / len;
    for (int i = 0; i < n; i += len) {
      for (int j = 0; j < half; ++j) {
        uint64_t u = a[i + j], v = mmul(a[i + j + half], wpow[j * step], q);
        a[i + j] = madd(u, v, q);
        a[i + j + half] = msub(u, v, q);
      }
    }
  }
}
/* forward: a(X) -> values a(psi * omega^k) in the cyclic transform's order */
static void ntt_fwd(orc_ctx* c, int t, uint64_t* a) {
  uint64_t q = c->mod[t];
  for (int i = 0; i < c->n; ++i) a[i] = mmul(a[i], c->psi_pow[t][i], q);
  cyclic_ntt(a, c->n, c->om_pow[t], q);
}
static void ntt_inv(orc_ctx* c, int t, uint64_t* a) {
  uint64_t q = c->mod[t];
  cyclic_ntt(a, c->n, c->om_ipow[t], q);
  for (int i = 0; i < c->n; ++i) a[i] = mmul(mmul(a[i], c->n_inv[t], q), c->psi_ipow[t][i], q);
}

/* ring product in Z_q[X]/(X^N+1), coefficient domain in and out */
static void ring_mul(orc_ctx* c, int t, const uint64_t* a, const uint64_t* b, uint64_t* out) {
  int n = c->n;
  uint64_t* x = (uint64_t*)xcalloc(n, 8);
  uint64_t* y = (uint64_t*)xcalloc(n, 8);
  memcpy(x, a, 8 * (size_t)n);
  memcpy(y, b, 8 * (size_t)n);
  ntt_fwd(c, t, x);
  ntt_fwd(c, t, y);
  for (int i = 0; i < n; ++i) x[i] = mmul(x[i], y[i], c->mod[t]);
  ntt_inv(c, t, x);
  memcpy(out, x, 8 * (size_t)n);
  free(x);
  free(y);
}

/* exported for the NTT pins: negacyclic product mod prime index t */
ORC_API void orc_ring_mul(void* h, int t, const uint64_t* a, const uint64_t* b, uint64_t* out) {
  ring_mul((orc_ctx*)h, t, a, b, out);
}
ORC_API void orc_ntt_roundtrip(void* h, int t, uint64_t* a) {
  orc_ctx* c = (orc_ctx*)h;
  ntt_fwd(c, t, a);
  ntt_inv(c, t, a);
}
ORC_API uint64_t orc_psi(void* h, int t) { orc_ctx* c = (orc_ctx*)h; return c->psi_pow[t][1]; }

/* ------------------------------------------------------------------------- */
/* ciphertexts                                                                */
/* ------------------------------------------------------------------------- */
typedef struct {
  int level;
  double scale;
  uint64_t* c[2]; /* (level+1) x N, coefficient domain, canonical residues */
} orc_ct;

static orc_ct* ct_new(orc_ctx* c, int level, double scale) {
  orc_ct* x = (orc_ct*)xcalloc(1, sizeof(orc_ct));
  x->level = level;
  x->scale = scale;
  for (int p = 0; p < 2; ++p) x->c[p] = (uint64_t*)xcalloc((size_t)(level + 1) * c->n, 8);
  return x;
}
static void ct_free(orc_ct* x) {
  if (!x) return;
  free(x->c[0]);
  free(x->c[1]);
  free(x);
}
static orc_ct* ct_copy(orc_ctx* c, const orc_ct* a, int level) {
  if (level > a->level) die("ct_copy: cannot raise level");
  orc_ct* x = ct_new(c, level, a->scale);
  for (int p = 0; p < 2; ++p) memcpy(x->c[p], a->c[p], 8 * (size_t)(level + 1) * c->n);
  return x;
}
#define LIMB(ct, p, i, n) ((ct)->c[p] + (size_t)(i) * (n))

ORC_API void* orc_ct_import(void* h, const uint64_t* data, int level, double scale) {
  orc_ctx* c = (orc_ctx*)h;
  orc_ct* x = ct_new(c, level, scale);
  size_t sz = (size_t)(level + 1) * c->n;
  memcpy(x->c[0], data, 8 * sz);
  memcpy(x->c[1], data + sz, 8 * sz);
  return x;
}
ORC_API void orc_ct_export(void* h, const void* ctp, uint64_t* data) {
  orc_ctx* c = (orc_ctx*)h;
  const orc_ct* x = (const orc_ct*)ctp;
  size_t sz = (size_t)(x->level + 1) * c->n;
  memcpy(data, x->c[0], 8 * sz);
  memcpy(data + sz, x->c[1], 8 * sz);
}
ORC_API int orc_ct_level(const void* x) { return ((const orc_ct*)x)->level; }
ORC_API double orc_ct_scale(const void* x) { return ((const orc_ct*)x)->scale; }
ORC_API void orc_ct_free(void* x) { ct_free((orc_ct*)x); }

/* ------------------------------------------------------------------------- */
/* encoding: canonical embedding on the slots j <-> root zeta^(5^j)           */
/* ------------------------------------------------------------------------- */
static int64_t round_half_away_q(__float128 x) {
  __float128 r = x >= 0 ? floorq(x + 0.5Q) : -floorq(-x + 0.5Q);
  if (fabsq(r) > 9.2e18Q) die("encode: coefficient exceeds int64");
  return (int64_t)r;
}
/* m_k = round(scale * 2/N * sum_j z_j cos(pi * (5^j * k mod 2N) / N)) for real slot values */
static void encode_real(orc_ctx* c, const double* z, int nslots, double scale, int64_t* m) {
  int n = c->n;
  uint64_t m2n = 2ull * (uint64_t)n;
  __float128 f = (__float128)scale * 2 / (__float128)n;
  for (int k = 0; k < n; ++k) {
    __float128 acc = 0;
    for (int j = 0; j < nslots; ++j) {
      if (z[j] == 0.0) continue;
      uint64_t t = (c->rot_group[j] * (uint64_t)k) % m2n;
      acc += (__float128)z[j] * c->cos_tab[t];
    }
    m[k] = round_half_away_q(f * acc);
  }
}
ORC_API void orc_encode(void* h, const double* z, int nslots, double scale, int64_t* m) {
  encode_real((orc_ctx*)h, z, nslots, scale, m);
}
/* real part of slot j: (1/scale) * sum_k m_k cos(pi * (5^j k mod 2N)/N) */
static void decode_real(orc_ctx* c, const i128* m, double scale, int nslots, double* z) {
  int n = c->n;
  uint64_t m2n = 2ull * (uint64_t)n;
  for (int j = 0; j < nslots; ++j) {
    __float128 acc = 0;
    for (int k = 0; k < n; ++k) {
      if (m[k] == 0) continue;
      uint64_t t = (c->rot_group[j] * (uint64_t)k) % m2n;
      acc += (__float128)m[k] * c->cos_tab[t];
    }
    z[j] = (double)(acc / (__float128)scale);
  }
}
ORC_API void orc_decode(void* h, const int64_t* m, double scale, int nslots, double* z) {
  orc_ctx* c = (orc_ctx*)h;
  i128* w = (i128*)xcalloc(c->n, sizeof(i128));
  for (int k = 0; k < c->n; ++k) w[k] = m[k];
  decode_real(c, w, scale, nslots, z);
  free(w);
}

/* ------------------------------------------------------------------------- */
/* key generation                                                             */
/* ------------------------------------------------------------------------- */
static void poly_from_small(orc_ctx* c, const int64_t* v, int t, uint64_t* out) {
  for (int i = 0; i < c->n; ++i) out[i] = from_i128(v[i], c->mod[t]);
}

ORC_API void orc_gen_secret(void* h, uint64_t seed) {
  orc_ctx* c = (orc_ctx*)h;
  free(c->s);
  c->s = (int64_t*)xcalloc(c->n, sizeof(int64_t));
  uint64_t key = sm_key(seed, make_tag(PUR_SECRET, 0, 0, LIMB_NONE));
  for (int i = 0; i < c->n; ++i)
    c->s[i] = c->secret_h > 0 ? sample_sparse(key, (uint64_t)i, c->log_n, c->secret_h) : sample_ternary(key, (uint64_t)i);
}
ORC_API void orc_get_secret(void* h, int64_t* out) { orc_ctx* c = (orc_ctx*)h; memcpy(out, c->s, 8 * (size_t)c->n); }

/* sigma_g on an integer polynomial: X^i -> X^(i g mod 2N) with X^N = -1 */
static void automorph_small(orc_ctx* c, const int64_t* in, uint64_t g, int64_t* out) {
  uint64_t n = (uint64_t)c->n;
  for (uint64_t i = 0; i < n; ++i) {
    uint64_t j = (i * g) % (2 * n);
    if (j < n) out[j] = in[i];
    else out[j - n] = -in[i];
  }
}
static void automorph_mod(orc_ctx* c, const uint64_t* in, uint64_t g, uint64_t q, uint64_t* out) {
  uint64_t n = (uint64_t)c->n;
  for (uint64_t i = 0; i < n; ++i) {
    uint64_t j = (i * g) % (2 * n);
    if (j < n) out[j] = in[i];
    else out[j - n] = mneg(in[i], q);
  }
}

/* P mod q_t, product of the special primes */
static uint64_t p_mod(orc_ctx* c, int t) {
  uint64_t r = 1 % c->mod[t];
  for (int k = 0; k < c->n_p; ++k) r = mmul(r, c->mod[c->n_q + k] % c->mod[t], c->mod[t]);
  return r;
}

/* switching key for s' -> s: per digit j (alpha consecutive chain primes at the
   top level), b_j = -a_j s + e_j + P * T_j * s' (mod QP), T_j = 1 mod primes of
   digit j and 0 mod the other chain primes. Stored in the NTT domain. */
static void gen_switch_key(orc_ctx* c, orc_key* k, const int64_t* s_from, uint64_t seed, int purpose, uint64_t obj) {
  int np = c->n_q + c->n_p, n = c->n;
  k->b = (uint64_t***)xcalloc(c->dnum, sizeof(uint64_t**));
  k->a = (uint64_t***)xcalloc(c->dnum, sizeof(uint64_t**));
  uint64_t* sm = (uint64_t*)xcalloc(n, 8);
  uint64_t* tmp = (uint64_t*)xcalloc(n, 8);
  int64_t* e = (int64_t*)xcalloc(n, 8);
  for (int j = 0; j < c->dnum; ++j) {
    k->b[j] = (uint64_t**)xcalloc(np, sizeof(uint64_t*));
    k->a[j] = (uint64_t**)xcalloc(np, sizeof(uint64_t*));
    uint64_t ekey = sm_key(seed, make_tag((uint64_t)purpose, obj, (uint64_t)j, LIMB_NONE));
    for (int i = 0; i < n; ++i) e[i] = sample_cbd21(ekey, (uint64_t)i);
    for (int t = 0; t < np; ++t) {
      uint64_t q = c->mod[t];
      uint64_t* a = (uint64_t*)xcalloc(n, 8);
      uint64_t* b = (uint64_t*)xcalloc(n, 8);
      uint64_t akey = sm_key(seed, make_tag((uint64_t)purpose, obj, (uint64_t)j, (uint64_t)t));
      for (int i = 0; i < n; ++i) a[i] = sample_uniform(akey, (uint64_t)i, q);
      poly_from_small(c, c->s, t, sm);
      ring_mul(c, t, a, sm, tmp);
      int in_digit = t < c->n_q && t / c->alpha == j;
      uint64_t pq = in_digit ? p_mod(c, t) : 0;
      for (int i = 0; i < n; ++i) {
        uint64_t v = msub(from_i128(e[i], q), tmp[i], q);
        if (in_digit) v = madd(v, mmul(pq, from_i128(s_from[i], q), q), q);
        b[i] = v;
      }
      ntt_fwd(c, t, a);
      ntt_fwd(c, t, b);
      k->a[j][t] = a;
      k->b[j][t] = b;
    }
  }
  free(sm);
  free(tmp);
  free(e);
}

static orc_key* find_key(orc_ctx* c, uint64_t g) {
  for (int i = 0; i < c->n_keys; ++i)
    if (c->keys[i].g == g) return &c->keys[i];
  return NULL;
}
static orc_key* add_key(orc_ctx* c, uint64_t g) {
  orc_key* old = find_key(c, g);
  if (old) { free_key(c, old); return old; }
  c->keys = (orc_key*)realloc(c->keys, sizeof(orc_key) * (size_t)(c->n_keys + 1));
  orc_key* k = &c->keys[c->n_keys++];
  memset(k, 0, sizeof(*k));
  k->g = g;
  return k;
}

/* the step value that asks for the conjugation X -> X^(2N-1) */
#define CONJ_STEP INT64_MIN
static uint64_t galois_elt(orc_ctx* c, int64_t step) {
  if (step == CONJ_STEP) return 2ull * (uint64_t)c->n - 1;
  int64_t slots = c->n / 2;
  int64_t r = ((step % slots) + slots) % slots;
  return c->rot_group[r];
}

/* s is generated from the same seed; rotation keys for RotL(step) */
ORC_API void orc_keygen(void* h, uint64_t seed, const int64_t* steps, int n_steps) {
  orc_ctx* c = (orc_ctx*)h;
  int n = c->n;
  orc_gen_secret(h, seed);
  /* relinearisation: s^2 -> s.  The coefficients of s^2 in Z[X]/(X^N+1) are
     bounded by N < q_0/2, so the ring product mod q_0 lifted to (-q_0/2, q_0/2]
     is s^2 itself. */
  int64_t* s2 = (int64_t*)xcalloc(n, 8);
  {
    uint64_t q0 = c->mod[0];
    uint64_t* sq = (uint64_t*)xcalloc(n, 8);
    uint64_t* pr = (uint64_t*)xcalloc(n, 8);
    poly_from_small(c, c->s, 0, sq);
    ring_mul(c, 0, sq, sq, pr);
    for (int i = 0; i < n; ++i) s2[i] = pr[i] > q0 / 2 ? (int64_t)pr[i] - (int64_t)q0 : (int64_t)pr[i];
    free(sq);
    free(pr);
  }
  orc_key* rk = add_key(c, 0);
  rk->g = 0;
  gen_switch_key(c, rk, s2, seed, PUR_RELIN, 0);
  free(s2);
  int64_t* sg = (int64_t*)xcalloc(n, 8);
  for (int i = 0; i < n_steps; ++i) {
    uint64_t g = galois_elt(c, steps[i]);
    if (g == 1 || find_key(c, g)) continue;
    automorph_small(c, c->s, g, sg);
    orc_key* k = add_key(c, g);
    gen_switch_key(c, k, sg, seed, PUR_GALOIS, g);
  }
  free(sg);
}

/* key limb in the coefficient domain (for parity checks) */
ORC_API int orc_get_key(void* h, uint64_t g, int digit, int which, int t, uint64_t* out) {
  orc_ctx* c = (orc_ctx*)h;
  orc_key* k = find_key(c, g);
  if (!k || digit >= c->dnum || t >= c->n_q + c->n_p) return -1;
  memcpy(out, which ? k->a[digit][t] : k->b[digit][t], 8 * (size_t)c->n);
  ntt_inv(c, t, out);
  return 0;
}

/* ------------------------------------------------------------------------- */
/* encryption / decryption                                                    */
/* ------------------------------------------------------------------------- */
/* secret-key encryption of integer plaintext m at level 'level' */
static orc_ct* encrypt_int(orc_ctx* c, const i128* m, double scale, uint64_t seed, int purpose, uint64_t sub, int level) {
  if (!c->s) die("encrypt: no secret (keygen first)");
  int n = c->n;
  orc_ct* x = ct_new(c, level, scale);
  uint64_t ekey = sm_key(seed, make_tag((uint64_t)purpose, 0, sub, LIMB_NONE));
  int64_t* e = (int64_t*)xcalloc(n, 8);
  for (int i = 0; i < n; ++i) e[i] = sample_cbd21(ekey, (uint64_t)i);
  uint64_t* sm = (uint64_t*)xcalloc(n, 8);
  uint64_t* as = (uint64_t*)xcalloc(n, 8);
  for (int t = 0; t <= level; ++t) {
    uint64_t q = c->mod[t];
    uint64_t* a = LIMB(x, 1, t, n);
    uint64_t akey = sm_key(seed, make_tag((uint64_t)purpose, 0, sub, (uint64_t)t));
    for (int i = 0; i < n; ++i) a[i] = sample_uniform(akey, (uint64_t)i, q);
    poly_from_small(c, c->s, t, sm);
    ring_mul(c, t, a, sm, as);
    uint64_t* b = LIMB(x, 0, t, n);
    for (int i = 0; i < n; ++i) b[i] = madd(msub(from_i128(m[i], q), as[i], q), from_i128(e[i], q), q);
  }
  free(e);
  free(sm);
  free(as);
  return x;
}

ORC_API void* orc_encrypt(void* h, const int64_t* m, double scale, uint64_t seed) {
  orc_ctx* c = (orc_ctx*)h;
  i128* w = (i128*)xcalloc(c->n, sizeof(i128));
  for (int i = 0; i < c->n; ++i) w[i] = m[i];
  orc_ct* x = encrypt_int(c, w, scale, seed, PUR_ENCRYPT, 0, c->n_q - 1);
  free(w);
  return x;
}

/* m = c0 + c1 s, lifted to the centred integer from limbs 0 and 1 (CRT) */
static void decrypt_int(orc_ctx* c, const orc_ct* x, i128* m) {
  int n = c->n;
  if (x->level < 1) die("decrypt needs at least two limbs");
  uint64_t* sm = (uint64_t*)xcalloc(n, 8);
  uint64_t* r[2];
  for (int t = 0; t < 2; ++t) {
    uint64_t q = c->mod[t];
    r[t] = (uint64_t*)xcalloc(n, 8);
    poly_from_small(c, c->s, t, sm);
    ring_mul(c, t, LIMB(x, 1, t, n), sm, r[t]);
    const uint64_t* b = LIMB(x, 0, t, n);
    for (int i = 0; i < n; ++i) r[t][i] = madd(r[t][i], b[i], q);
  }
  uint64_t q0 = c->mod[0], q1 = c->mod[1];
  uint64_t q0inv = minv(q0 % q1, q1);
  i128 Q = (i128)q0 * (i128)q1;
  for (int i = 0; i < n; ++i) {
    /* x = r0 + q0 * ((r1 - r0) q0^-1 mod q1), in [0, q0 q1) */
    uint64_t d = mmul(msub(r[1][i], r[0][i] % q1, q1), q0inv, q1);
    i128 v = (i128)r[0][i] + (i128)q0 * (i128)d;
    if (v > Q / 2) v -= Q;
    m[i] = v;
  }
  free(sm);
  free(r[0]);
  free(r[1]);
}

ORC_API void orc_decrypt(void* h, const void* ctp, int64_t* m_out) {
  orc_ctx* c = (orc_ctx*)h;
  i128* m = (i128*)xcalloc(c->n, sizeof(i128));
  decrypt_int(c, (const orc_ct*)ctp, m);
  for (int i = 0; i < c->n; ++i) {
    if (m[i] > (i128)INT64_MAX || m[i] < (i128)INT64_MIN) die("decrypt: message exceeds int64");
    m_out[i] = (int64_t)m[i];
  }
  free(m);
}

ORC_API void orc_decrypt_decode(void* h, const void* ctp, int nslots, double* z) {
  orc_ctx* c = (orc_ctx*)h;
  const orc_ct* x = (const orc_ct*)ctp;
  i128* m = (i128*)xcalloc(c->n, sizeof(i128));
  decrypt_int(c, x, m);
  decode_real(c, m, x->scale, nslots, z);
  free(m);
}

/* ------------------------------------------------------------------------- */
/* homomorphic operations                                                     */
/* ------------------------------------------------------------------------- */
static void check_scales(double a, double b) {
  if (fabs(a - b) > 1e-9 * fabs(a)) die("scale mismatch in addition");
}

static orc_ct* op_add(orc_ctx* c, const orc_ct* a, const orc_ct* b, int sub) {
  check_scales(a->scale, b->scale);
  int lvl = a->level < b->level ? a->level : b->level;
  orc_ct* x = ct_new(c, lvl, a->scale);
  int n = c->n;
  for (int p = 0; p < 2; ++p)
    for (int t = 0; t <= lvl; ++t) {
      uint64_t q = c->mod[t];
      const uint64_t* u = LIMB(a, p, t, n);
      const uint64_t* v = LIMB(b, p, t, n);
      uint64_t* w = LIMB(x, p, t, n);
      for (int i = 0; i < n; ++i) w[i] = sub ? msub(u[i], v[i], q) : madd(u[i], v[i], q);
    }
  return x;
}

/* add the real constant v to every slot: K = llround(v * scale) added to coefficient 0 */
static void op_add_const_inplace(orc_ctx* c, orc_ct* x, double v) {
  double kf = v * x->scale;
  int64_t K = llround(kf);
  for (int t = 0; t <= x->level; ++t) {
    uint64_t q = c->mod[t];
    uint64_t* w = LIMB(x, 0, t, c->n);
    w[0] = madd(w[0], from_i128(K, q), q);
  }
}

static void rescale_inplace(orc_ctx* c, orc_ct* x) {
  int l = x->level, n = c->n;
  if (l < 1) die("rescale at level 0");
  uint64_t ql = c->mod[l];
  for (int p = 0; p < 2; ++p) {
    const uint64_t* top = LIMB(x, p, l, n);
    for (int t = 0; t < l; ++t) {
      uint64_t q = c->mod[t];
      uint64_t inv = minv(ql % q, q);
      uint64_t* w = LIMB(x, p, t, n);
      for (int i = 0; i < n; ++i) {
        i128 r = top[i] > ql / 2 ? (i128)top[i] - (i128)ql : (i128)top[i];
        w[i] = mmul(msub(w[i], from_i128(r, q), q), inv, q);
      }
    }
  }
  x->level = l - 1;
  x->scale = x->scale / (double)ql;
}

/* constant multiply with exact target scale: K = llround(v * T * q_l / s), then
   rescale; the result is defined to carry scale T */
static orc_ct* op_lincomb(orc_ctx* c, const orc_ct* a, double va, const orc_ct* b, double vb, double target,
                          int rescale);
static orc_ct* op_mul_const(orc_ctx* c, const orc_ct* a, double v, double target) {
  return op_lincomb(c, a, v, NULL, 0.0, target, 1);
}

/* multiply by the encoded real vector v (nslots values) with exact target scale */
static orc_ct* op_mul_plain(orc_ctx* c, const orc_ct* a, const double* v, int nslots, double target) {
  int n = c->n;
  double ql = (double)c->mod[a->level];
  double pscale = target * ql;
  pscale = pscale / a->scale;
  int64_t* m = (int64_t*)xcalloc(n, 8);
  encode_real(c, v, nslots, pscale, m);
  orc_ct* x = ct_new(c, a->level, a->scale);
  uint64_t* mp = (uint64_t*)xcalloc(n, 8);
  for (int t = 0; t <= a->level; ++t) {
    poly_from_small(c, m, t, mp);
    for (int p = 0; p < 2; ++p) ring_mul(c, t, LIMB(a, p, t, n), mp, LIMB(x, p, t, n));
  }
  free(m);
  free(mp);
  rescale_inplace(c, x);
  x->scale = target;
  return x;
}

/* x = a + encode(v) at a's scale (the plaintext added to c0) */
static orc_ct* op_add_plain(orc_ctx* c, const orc_ct* a, const double* v, int nslots) {
  int n = c->n;
  int64_t* m = (int64_t*)xcalloc(n, 8);
  encode_real(c, v, nslots, a->scale, m);
  orc_ct* x = ct_copy(c, a, a->level);
  for (int t = 0; t <= x->level; ++t) {
    uint64_t q = c->mod[t];
    uint64_t* w = LIMB(x, 0, t, n);
    for (int i = 0; i < n; ++i) w[i] = madd(w[i], from_i128(m[i], q), q);
  }
  free(m);
  return x;
}

static uint64_t** alloc_limbs(int count, int n) {
  uint64_t** a = (uint64_t**)xcalloc(count, sizeof(uint64_t*));
  for (int e = 0; e < count; ++e) a[e] = (uint64_t*)xcalloc(n, 8);
  return a;
}
static void free_limbs(uint64_t** a, int count) {
  for (int e = 0; e < count; ++e) free(a[e]);
  free(a);
}

/* ModUp of hybrid key switching: d (coefficient domain, limbs 0..l) split
   into digits of alpha chain primes, each digit raised to Q_l u P (limbs
   0..l, then the special primes).  ext[j][e] is digit j on extended limb e,
   in the coefficient domain; on the digit's own primes it is d itself. */
static uint64_t*** modup_digits(orc_ctx* c, const uint64_t* d, int l, int* dn_out) {
  int n = c->n, alpha = c->alpha, n_q = c->n_q, n_p = c->n_p;
  int n_ext = l + 1 + n_p;
  int dn = (l + 1 + alpha - 1) / alpha;
  uint64_t*** ext = (uint64_t***)xcalloc(dn, sizeof(uint64_t**));
  for (int j = 0; j < dn; ++j) {
    int lo = j * alpha, hi = (j + 1) * alpha < l + 1 ? (j + 1) * alpha : l + 1;
    int sz = hi - lo;
    /* y_i = [d_i * (D/q_i)^{-1}]_{q_i} for i in the digit */
    uint64_t** y = (uint64_t**)xcalloc(sz, sizeof(uint64_t*));
    for (int i = 0; i < sz; ++i) {
      uint64_t qi = c->mod[lo + i];
      uint64_t dhat = 1;
      for (int i2 = 0; i2 < sz; ++i2)
        if (i2 != i) dhat = mmul(dhat, c->mod[lo + i2] % qi, qi);
      uint64_t inv = minv(dhat, qi);
      y[i] = (uint64_t*)xcalloc(n, 8);
      const uint64_t* di = d + (size_t)(lo + i) * n;
      for (int x = 0; x < n; ++x) y[i][x] = mmul(di[x], inv, qi);
    }
    ext[j] = alloc_limbs(n_ext, n);
    for (int e = 0; e < n_ext; ++e) {
      int t = e <= l ? e : n_q + (e - l - 1);
      uint64_t q = c->mod[t];
      uint64_t* limb = ext[j][e];
      if (t >= lo && t < hi) {
        memcpy(limb, d + (size_t)t * n, 8 * (size_t)n);
      } else {
        for (int i = 0; i < sz; ++i) {
          uint64_t dhat = 1; /* (D/q_i) mod q */
          for (int i2 = 0; i2 < sz; ++i2)
            if (i2 != i) dhat = mmul(dhat, c->mod[lo + i2] % q, q);
          for (int x = 0; x < n; ++x) limb[x] = madd(limb[x], mmul(y[i][x] % q, dhat, q), q);
        }
      }
    }
    for (int i = 0; i < sz; ++i) free(y[i]);
    free(y);
  }
  *dn_out = dn;
  return ext;
}
static void free_digits(uint64_t*** ext, int dn, int n_ext) {
  for (int j = 0; j < dn; ++j) free_limbs(ext[j], n_ext);
  free(ext);
}

/* inner product of the raised digits with key k, every digit limb first
   taken through X -> X^g (g = 1: unchanged), over Q_l u P:
   acc0 + acc1 s = P sigma_g(d) s' + small, returned in the coefficient domain */
static void ks_inner(orc_ctx* c, uint64_t*** ext, int dn, int l, uint64_t g, const orc_key* k, uint64_t** acc0,
                     uint64_t** acc1) {
  int n = c->n, n_q = c->n_q, n_p = c->n_p;
  int n_ext = l + 1 + n_p;
  uint64_t* limb = (uint64_t*)xcalloc(n, 8);
  for (int j = 0; j < dn; ++j) {
    for (int e = 0; e < n_ext; ++e) {
      int t = e <= l ? e : n_q + (e - l - 1);
      uint64_t q = c->mod[t];
      if (g == 1) memcpy(limb, ext[j][e], 8 * (size_t)n);
      else automorph_mod(c, ext[j][e], g, q, limb);
      ntt_fwd(c, t, limb);
      for (int x = 0; x < n; ++x) {
        acc0[e][x] = madd(acc0[e][x], mmul(limb[x], k->b[j][t][x], q), q);
        acc1[e][x] = madd(acc1[e][x], mmul(limb[x], k->a[j][t][x], q), q);
      }
    }
  }
  for (int e = 0; e < n_ext; ++e) {
    int t = e <= l ? e : n_q + (e - l - 1);
    ntt_inv(c, t, acc0[e]);
    ntt_inv(c, t, acc1[e]);
  }
  free(limb);
  c->counters[CNT_KS]++;
}

/* first half of the hybrid key switch of d (coefficient domain, limbs 0..l)
   with key k: ModUp of every digit and the inner product with the key,
   returned in the coefficient domain over Q_l u P (limbs 0..l, then the
   special primes): acc0 + acc1 s = P d s' + small  (mod Q_l P) */
static void key_switch_raw(orc_ctx* c, const uint64_t* d, int l, const orc_key* k, uint64_t** acc0, uint64_t** acc1) {
  int dn;
  uint64_t*** ext = modup_digits(c, d, l, &dn);
  ks_inner(c, ext, dn, l, 1, k, acc0, acc1);
  free_digits(ext, dn, l + 1 + c->n_p);
}

/* z in [0, b) read as its centred representative in (-b/2, b/2), reduced mod q */
static uint64_t centred_mod(uint64_t z, uint64_t b, uint64_t q) {
  if (z <= b / 2) return z % q;
  uint64_t m = (b - z) % q;
  return m ? q - m : 0;
}


/* ModDown of hybrid key switching: (acc0, acc1) over Q_l u P (coefficient
   domain) divided by P with rounding -> (u0, u1) in R_{Q_l}; frees acc0, acc1 */
static void mod_down(orc_ctx* c, uint64_t** acc0, uint64_t** acc1, int l, uint64_t* u0, uint64_t* u1) {
  int n = c->n, n_q = c->n_q, n_p = c->n_p;
  int n_ext = l + 1 + n_p;
  /* ModDown: (u - Conv_{P->q}([u]_P)) * P^{-1} mod q, the conversion taking
     each [u (P/p)^{-1}]_p centred so the division rounds without bias */
  for (int which = 0; which < 2; ++which) {
    uint64_t** acc = which ? acc1 : acc0;
    uint64_t* out = which ? u1 : u0;
    uint64_t** y = (uint64_t**)xcalloc(n_p, sizeof(uint64_t*));
    for (int kp = 0; kp < n_p; ++kp) {
      uint64_t pk = c->mod[n_q + kp];
      uint64_t phat = 1;
      for (int k2 = 0; k2 < n_p; ++k2)
        if (k2 != kp) phat = mmul(phat, c->mod[n_q + k2] % pk, pk);
      uint64_t inv = minv(phat, pk);
      y[kp] = (uint64_t*)xcalloc(n, 8);
      for (int x = 0; x < n; ++x) y[kp][x] = mmul(acc[l + 1 + kp][x], inv, pk);
    }
    for (int t = 0; t <= l; ++t) {
      uint64_t q = c->mod[t];
      uint64_t pinv = minv(p_mod(c, t), q);
      uint64_t* o = out + (size_t)t * n;
      for (int x = 0; x < n; ++x) o[x] = 0;
      for (int kp = 0; kp < n_p; ++kp) {
        uint64_t phat = 1;
        for (int k2 = 0; k2 < n_p; ++k2)
          if (k2 != kp) phat = mmul(phat, c->mod[n_q + k2] % q, q);
        for (int x = 0; x < n; ++x) o[x] = madd(o[x], mmul(centred_mod(y[kp][x], c->mod[n_q + kp], q), phat, q), q);
      }
      for (int x = 0; x < n; ++x) o[x] = mmul(msub(acc[t][x], o[x], q), pinv, q);
    }
    for (int kp = 0; kp < n_p; ++kp) free(y[kp]);
    free(y);
  }
  free_limbs(acc0, n_ext);
  free_limbs(acc1, n_ext);
}

/* hybrid key switch of d (coefficient domain, limbs 0..l) with key k:
   returns (u0, u1) in R_{Q_l} with u0 + u1 s ~ d s' */
static void key_switch(orc_ctx* c, const uint64_t* d, int l, const orc_key* k, uint64_t* u0, uint64_t* u1) {
  int n_ext = l + 1 + c->n_p;
  uint64_t** acc0 = alloc_limbs(n_ext, c->n);
  uint64_t** acc1 = alloc_limbs(n_ext, c->n);
  key_switch_raw(c, d, l, k, acc0, acc1);
  mod_down(c, acc0, acc1, l, u0, u1);
}

/* ct x ct: tensor, relinearise (key switch of the s^2 part); caller rescales */
static orc_ct* op_mul_relin(orc_ctx* c, const orc_ct* a_in, const orc_ct* b_in) {
  int l = a_in->level < b_in->level ? a_in->level : b_in->level;
  int n = c->n;
  orc_key* rk = find_key(c, 0);
  if (!rk) die("no relinearisation key");
  orc_ct* x = ct_new(c, l, a_in->scale * b_in->scale);
  uint64_t* d2 = (uint64_t*)xcalloc((size_t)(l + 1) * n, 8);
  uint64_t *a0 = (uint64_t*)xcalloc(n, 8), *a1 = (uint64_t*)xcalloc(n, 8);
  uint64_t *b0 = (uint64_t*)xcalloc(n, 8), *b1 = (uint64_t*)xcalloc(n, 8);
  for (int t = 0; t <= l; ++t) {
    uint64_t q = c->mod[t];
    memcpy(a0, LIMB(a_in, 0, t, n), 8 * (size_t)n);
    memcpy(a1, LIMB(a_in, 1, t, n), 8 * (size_t)n);
    memcpy(b0, LIMB(b_in, 0, t, n), 8 * (size_t)n);
    memcpy(b1, LIMB(b_in, 1, t, n), 8 * (size_t)n);
    ntt_fwd(c, t, a0); ntt_fwd(c, t, a1); ntt_fwd(c, t, b0); ntt_fwd(c, t, b1);
    uint64_t* x0 = LIMB(x, 0, t, n);
    uint64_t* x1 = LIMB(x, 1, t, n);
    uint64_t* x2 = d2 + (size_t)t * n;
    for (int i = 0; i < n; ++i) {
      x0[i] = mmul(a0[i], b0[i], q);
      x1[i] = madd(mmul(a0[i], b1[i], q), mmul(a1[i], b0[i], q), q);
      x2[i] = mmul(a1[i], b1[i], q);
    }
    ntt_inv(c, t, x0); ntt_inv(c, t, x1); ntt_inv(c, t, x2);
  }
  free(a0); free(a1); free(b0); free(b1);
  uint64_t* u0 = (uint64_t*)xcalloc((size_t)(l + 1) * n, 8);
  uint64_t* u1 = (uint64_t*)xcalloc((size_t)(l + 1) * n, 8);
  key_switch(c, d2, l, rk, u0, u1);
  for (int t = 0; t <= l; ++t) {
    uint64_t q = c->mod[t];
    for (int i = 0; i < n; ++i) {
      size_t o = (size_t)t * n + i;
      x->c[0][o] = madd(x->c[0][o], u0[o], q);
      x->c[1][o] = madd(x->c[1][o], u1[o], q);
    }
  }
  free(d2); free(u0); free(u1);
  c->counters[CNT_RELIN]++;
  return x;
}

/* a degree-2 ciphertext (d0, d1, d2), coefficient domain, decrypting as d0 + d1 s + d2 s^2 */
typedef struct {
  int level;
  double scale;
  uint64_t* c[3];
} orc_ct3;

static orc_ct3* ct3_new(orc_ctx* c, int level, double scale) {
  orc_ct3* x = (orc_ct3*)xcalloc(1, sizeof(orc_ct3));
  x->level = level;
  x->scale = scale;
  for (int p = 0; p < 3; ++p) x->c[p] = (uint64_t*)xcalloc((size_t)(level + 1) * c->n, 8);
  return x;
}
static void ct3_free(orc_ct3* x) {
  if (!x) return;
  for (int p = 0; p < 3; ++p) free(x->c[p]);
  free(x);
}

/* tensor product: (a0 + a1 s)(b0 + b1 s) = a0 b0 + (a0 b1 + a1 b0) s + a1 b1 s^2 */
static orc_ct3* op_tensor(orc_ctx* c, const orc_ct* a, const orc_ct* b) {
  int l = a->level < b->level ? a->level : b->level;
  int n = c->n;
  orc_ct3* x = ct3_new(c, l, a->scale * b->scale);
  uint64_t* t = (uint64_t*)xcalloc(n, 8);
  for (int i = 0; i <= l; ++i) {
    uint64_t q = c->mod[i];
    ring_mul(c, i, LIMB(a, 0, i, n), LIMB(b, 0, i, n), x->c[0] + (size_t)i * n);
    ring_mul(c, i, LIMB(a, 0, i, n), LIMB(b, 1, i, n), x->c[1] + (size_t)i * n);
    ring_mul(c, i, LIMB(a, 1, i, n), LIMB(b, 0, i, n), t);
    uint64_t* d1 = x->c[1] + (size_t)i * n;
    for (int k = 0; k < n; ++k) d1[k] = madd(d1[k], t[k], q);
    ring_mul(c, i, LIMB(a, 1, i, n), LIMB(b, 1, i, n), x->c[2] + (size_t)i * n);
  }
  free(t);
  return x;
}

/* x += y (degree-2 + degree-2); levels must match */
static void op_add3_inplace(orc_ctx* c, orc_ct3* x, const orc_ct3* y) {
  check_scales(x->scale, y->scale);
  if (x->level != y->level) die("op_add3: level mismatch");
  for (int p = 0; p < 3; ++p)
    for (int i = 0; i <= x->level; ++i) {
      uint64_t q = c->mod[i];
      uint64_t* u = x->c[p] + (size_t)i * c->n;
      const uint64_t* v = y->c[p] + (size_t)i * c->n;
      for (int k = 0; k < c->n; ++k) u[k] = madd(u[k], v[k], q);
    }
}

/* x += a (a degree-1 ciphertext at x's level or above) */
static void op_add3_ct_inplace(orc_ctx* c, orc_ct3* x, const orc_ct* a) {
  check_scales(x->scale, a->scale);
  if (a->level < x->level) die("op_add3_ct: level");
  for (int p = 0; p < 2; ++p)
    for (int i = 0; i <= x->level; ++i) {
      uint64_t q = c->mod[i];
      uint64_t* u = x->c[p] + (size_t)i * c->n;
      const uint64_t* v = LIMB(a, p, i, c->n);
      for (int k = 0; k < c->n; ++k) u[k] = madd(u[k], v[k], q);
    }
}

/* Relinearise and rescale in one division.  With the key-switch accumulator
   acc of d2 over Q_l u P (acc0 + acc1 s = P d2 s^2 + small), form
   y_w = P d_w + acc_w over Q_l u P and divide exactly by P q_l:
     out_w = (y_w - Conv_{B -> Q_{l-1}}([y_w]_B)) (P q_l)^{-1},  B = {q_l} u P,
   Conv being the approximate base conversion with centred digits (as in
   ModDown), so out_w = round(y_w / (P q_l)) + v with |v| <= |B| / 2.  The
   result is (d0 + d1 s + d2 s^2) / q_l up to small unbiased rounding: one
   level down. */
static orc_ct* op_relin_rescale(orc_ctx* c, const orc_ct3* x) {
  int l = x->level, n = c->n, n_q = c->n_q, n_p = c->n_p;
  if (l < 1) die("relin_rescale at level 0");
  orc_key* rk = find_key(c, 0);
  if (!rk) die("no relinearisation key");
  int n_ext = l + 1 + n_p;
  uint64_t** acc[2] = {alloc_limbs(n_ext, n), alloc_limbs(n_ext, n)};
  key_switch_raw(c, x->c[2], l, rk, acc[0], acc[1]);
  /* base B: q_l then the special primes; b_idx = absolute prime index, e_idx = extended-basis index */
  int nb = n_p + 1;
  int* b_idx = (int*)xcalloc(nb, sizeof(int));
  int* e_idx = (int*)xcalloc(nb, sizeof(int));
  b_idx[0] = l;
  e_idx[0] = l;
  for (int k = 0; k < n_p; ++k) { b_idx[1 + k] = n_q + k; e_idx[1 + k] = l + 1 + k; }
  orc_ct* out = ct_new(c, l - 1, x->scale / (double)c->mod[l]);
  uint64_t* yb = (uint64_t*)xcalloc(n, 8);
  for (int w = 0; w < 2; ++w) {
    /* y over Q_l u P: P d_w + acc_w on the chain primes, acc_w on the special primes */
    for (int t = 0; t <= l; ++t) {
      uint64_t q = c->mod[t], pm = p_mod(c, t);
      const uint64_t* d = x->c[w] + (size_t)t * n;
      for (int k = 0; k < n; ++k) acc[w][t][k] = madd(mmul(pm, d[k], q), acc[w][t][k], q);
    }
    /* z_b = [y_b (B/b)^{-1}]_b */
    uint64_t** zb = alloc_limbs(nb, n);
    for (int i = 0; i < nb; ++i) {
      uint64_t qb = c->mod[b_idx[i]], bhat = 1;
      for (int i2 = 0; i2 < nb; ++i2)
        if (i2 != i) bhat = mmul(bhat, c->mod[b_idx[i2]] % qb, qb);
      uint64_t inv = minv(bhat, qb);
      for (int k = 0; k < n; ++k) zb[i][k] = mmul(acc[w][e_idx[i]][k], inv, qb);
    }
    for (int t = 0; t < l; ++t) {
      uint64_t q = c->mod[t];
      uint64_t Bq = 1;
      for (int i = 0; i < nb; ++i) Bq = mmul(Bq, c->mod[b_idx[i]] % q, q);
      uint64_t binv = minv(Bq, q);
      for (int k = 0; k < n; ++k) yb[k] = 0;
      for (int i = 0; i < nb; ++i) {
        uint64_t bhat = 1; /* (B/b_i) mod q */
        for (int i2 = 0; i2 < nb; ++i2)
          if (i2 != i) bhat = mmul(bhat, c->mod[b_idx[i2]] % q, q);
        for (int k = 0; k < n; ++k) yb[k] = madd(yb[k], mmul(centred_mod(zb[i][k], c->mod[b_idx[i]], q), bhat, q), q);
      }
      uint64_t* o = LIMB(out, w, t, n);
      for (int k = 0; k < n; ++k) o[k] = mmul(msub(acc[w][t][k], yb[k], q), binv, q);
    }
    free_limbs(zb, nb);
  }
  free(yb);
  free(b_idx);
  free(e_idx);
  free_limbs(acc[0], n_ext);
  free_limbs(acc[1], n_ext);
  c->counters[CNT_RELIN]++;
  return out;
}

static orc_ct* op_mul_relin_rescale(orc_ctx* c, const orc_ct* a, const orc_ct* b) {
  orc_ct3* t = op_tensor(c, a, b);
  orc_ct* x = op_relin_rescale(c, t);
  ct3_free(t);
  return x;
}

/* integer constant for value v taking scale s to T: llround(v T q / s) when a
   rescale by q follows, llround(v T / s) when none does */
static int64_t const_for(double v, double target, double q, double s, int rescale) {
  double k = v * target;
  if (rescale) k = k * q;
  k = k / s;
  if (!(fabs(k) < 9.2e18)) die("constant does not fit 64 bits");
  return llround(k);
}

/* K_a a + K_b b with integer constants chosen so the result carries scale T:
   rescaled once (rescale = 1) or left at the inputs' level (rescale = 0).
   b may be NULL; a and b share the level. */
static orc_ct* op_lincomb(orc_ctx* c, const orc_ct* a, double va, const orc_ct* b, double vb, double target,
                          int rescale) {
  int l = a->level, n = c->n;
  if (b && b->level != l) die("op_lincomb: level mismatch");
  double ql = (double)c->mod[l];
  int64_t Ka = const_for(va, target, ql, a->scale, rescale);
  int64_t Kb = b ? const_for(vb, target, ql, b->scale, rescale) : 0;
  orc_ct* x = ct_new(c, l, target);
  for (int p = 0; p < 2; ++p)
    for (int t = 0; t <= l; ++t) {
      uint64_t q = c->mod[t], kA = from_i128(Ka, q), kB = from_i128(Kb, q);
      const uint64_t* u = LIMB(a, p, t, n);
      const uint64_t* v = b ? LIMB(b, p, t, n) : NULL;
      uint64_t* w = LIMB(x, p, t, n);
      for (int k = 0; k < n; ++k) w[k] = b ? madd(mmul(u[k], kA, q), mmul(v[k], kB, q), q) : mmul(u[k], kA, q);
    }
  if (rescale) rescale_inplace(c, x);
  x->scale = target;
  return x;
}

/* automorphism X -> X^g, then key switch back to s */
static orc_ct* op_automorph_ks(orc_ctx* c, const orc_ct* a, uint64_t g) {
  if (g == 1) return ct_copy(c, a, a->level);
  orc_key* k = find_key(c, g);
  if (!k) die("missing Galois key");
  int l = a->level, n = c->n;
  orc_ct* x = ct_new(c, l, a->scale);
  uint64_t* d = (uint64_t*)xcalloc((size_t)(l + 1) * n, 8);
  for (int t = 0; t <= l; ++t) {
    automorph_mod(c, LIMB(a, 0, t, n), g, c->mod[t], LIMB(x, 0, t, n));
    automorph_mod(c, LIMB(a, 1, t, n), g, c->mod[t], d + (size_t)t * n);
  }
  uint64_t* u0 = (uint64_t*)xcalloc((size_t)(l + 1) * n, 8);
  key_switch(c, d, l, k, u0, x->c[1]);
  for (int t = 0; t <= l; ++t)
    for (int i = 0; i < n; ++i) {
      size_t o = (size_t)t * n + i;
      x->c[0][o] = madd(x->c[0][o], u0[o], c->mod[t]);
    }
  free(d);
  free(u0);
  c->counters[CNT_ROT]++;
  return x;
}
/* RotL(x, step): slot j <- slot j+step (g = 5^step); the conjugation for CONJ_STEP */
static orc_ct* op_rotate(orc_ctx* c, const orc_ct* a, int64_t step) { return op_automorph_ks(c, a, galois_elt(c, step)); }

/* hoisted rotations of one ciphertext by several steps: the ModUp of c1 is
   computed once and each rotation applies X -> X^g to the raised digits
   (a signed permutation of coefficients, exact on every limb) before its own
   inner product and ModDown.  The result differs from RotL's by the basis
   extension's overshoot, a multiple of the digit modulus, which the key
   switch divides by P like any other error. */
static void op_rotate_hoisted(orc_ctx* c, const orc_ct* a, const int64_t* steps, int m, orc_ct** out) {
  int l = a->level, n = c->n;
  int n_ext = l + 1 + c->n_p;
  int dn = 0;
  uint64_t*** ext = NULL;
  for (int s = 0; s < m; ++s) {
    uint64_t g = galois_elt(c, steps[s]);
    if (g == 1) {
      out[s] = ct_copy(c, a, l);
      continue;
    }
    orc_key* k = find_key(c, g);
    if (!k) die("missing Galois key");
    if (!ext) ext = modup_digits(c, a->c[1], l, &dn);
    orc_ct* x = ct_new(c, l, a->scale);
    uint64_t** acc0 = alloc_limbs(n_ext, n);
    uint64_t** acc1 = alloc_limbs(n_ext, n);
    ks_inner(c, ext, dn, l, g, k, acc0, acc1);
    uint64_t* u0 = (uint64_t*)xcalloc((size_t)(l + 1) * n, 8);
    mod_down(c, acc0, acc1, l, u0, x->c[1]);
    for (int t = 0; t <= l; ++t) {
      automorph_mod(c, LIMB(a, 0, t, n), g, c->mod[t], LIMB(x, 0, t, n));
      uint64_t* o = LIMB(x, 0, t, n);
      const uint64_t* u = u0 + (size_t)t * n;
      for (int i = 0; i < n; ++i) o[i] = madd(o[i], u[i], c->mod[t]);
    }
    free(u0);
    c->counters[CNT_ROT]++;
    out[s] = x;
  }
  if (ext) free_digits(ext, dn, n_ext);
}

/* key-owner refresh, the stand-in for bootstrapping: decrypt, lift the message
   exactly and re-encrypt at the top level with fresh randomness; scale kept */
static orc_ct* op_refresh(orc_ctx* c, const orc_ct* a, uint64_t seed, uint64_t index) {
  i128* m = (i128*)xcalloc(c->n, sizeof(i128));
  decrypt_int(c, a, m);
  orc_ct* x = encrypt_int(c, m, a->scale, seed, PUR_REFRESH, index, c->refresh_level);
  free(m);
  c->counters[CNT_REFRESH]++;
  return x;
}

/* exported primitive operations (handles in, new handle out) */
ORC_API void* orc_add(void* h, const void* a, const void* b) { return op_add((orc_ctx*)h, (const orc_ct*)a, (const orc_ct*)b, 0); }
ORC_API void* orc_sub(void* h, const void* a, const void* b) { return op_add((orc_ctx*)h, (const orc_ct*)a, (const orc_ct*)b, 1); }
ORC_API void* orc_add_const(void* h, const void* a, double v) {
  orc_ctx* c = (orc_ctx*)h;
  orc_ct* x = ct_copy(c, (const orc_ct*)a, ((const orc_ct*)a)->level);
  op_add_const_inplace(c, x, v);
  return x;
}
ORC_API void* orc_rescale(void* h, const void* a) {
  orc_ctx* c = (orc_ctx*)h;
  orc_ct* x = ct_copy(c, (const orc_ct*)a, ((const orc_ct*)a)->level);
  rescale_inplace(c, x);
  return x;
}
ORC_API void* orc_lower(void* h, const void* a, int level) { return ct_copy((orc_ctx*)h, (const orc_ct*)a, level); }
ORC_API void* orc_mul_const(void* h, const void* a, double v, double target) { return op_mul_const((orc_ctx*)h, (const orc_ct*)a, v, target); }
ORC_API void* orc_mul_plain(void* h, const void* a, const double* v, int nslots, double target) {
  return op_mul_plain((orc_ctx*)h, (const orc_ct*)a, v, nslots, target);
}
ORC_API void* orc_mul_relin(void* h, const void* a, const void* b) { return op_mul_relin((orc_ctx*)h, (const orc_ct*)a, (const orc_ct*)b); }
ORC_API void* orc_mul_relin_rescale(void* h, const void* a, const void* b) {
  return op_mul_relin_rescale((orc_ctx*)h, (const orc_ct*)a, (const orc_ct*)b);
}
ORC_API void* orc_rotate(void* h, const void* a, int64_t step) { return op_rotate((orc_ctx*)h, (const orc_ct*)a, step); }
/* hoisted rotations of a by steps[0..m): out[i] = RotL(a, steps[i]) sharing one ModUp */
ORC_API void orc_rotate_hoisted(void* h, const void* a, const int64_t* steps, int m, void** out) {
  op_rotate_hoisted((orc_ctx*)h, (const orc_ct*)a, steps, m, (orc_ct**)out);
}
ORC_API void* orc_refresh(void* h, const void* a, uint64_t seed, uint64_t index) {
  return op_refresh((orc_ctx*)h, (const orc_ct*)a, seed, index);
}
ORC_API void orc_key_switch(void* h, uint64_t g, const uint64_t* d, int level, uint64_t* u0, uint64_t* u1) {
  orc_ctx* c = (orc_ctx*)h;
  orc_key* k = find_key(c, g);
  if (!k) die("missing key");
  key_switch(c, d, level, k, u0, u1);
}
/* acc0, acc1: (level + 1 + n_p) x N, chain limbs then special limbs */
ORC_API void orc_key_switch_raw(void* h, uint64_t g, const uint64_t* d, int level, uint64_t* acc0, uint64_t* acc1) {
  orc_ctx* c = (orc_ctx*)h;
  orc_key* k = find_key(c, g);
  if (!k) die("missing key");
  int n_ext = level + 1 + c->n_p;
  uint64_t** a0 = alloc_limbs(n_ext, c->n);
  uint64_t** a1 = alloc_limbs(n_ext, c->n);
  key_switch_raw(c, d, level, k, a0, a1);
  for (int e = 0; e < n_ext; ++e) {
    memcpy(acc0 + (size_t)e * c->n, a0[e], 8 * (size_t)c->n);
    memcpy(acc1 + (size_t)e * c->n, a1[e], 8 * (size_t)c->n);
  }
  free_limbs(a0, n_ext);
  free_limbs(a1, n_ext);
}
/* d: 3 x (level + 1) x N, a degree-2 ciphertext in the coefficient domain */
ORC_API void* orc_relin_rescale3(void* h, const uint64_t* d, int level, double scale) {
  orc_ctx* c = (orc_ctx*)h;
  orc_ct3* x = ct3_new(c, level, scale);
  for (int p = 0; p < 3; ++p) memcpy(x->c[p], d + (size_t)p * (level + 1) * c->n, 8 * (size_t)(level + 1) * c->n);
  orc_ct* y = op_relin_rescale(c, x);
  ct3_free(x);
  return y;
}
ORC_API void* orc_lincomb(void* h, const void* a, double va, const void* b, double vb, double target, int rescale) {
  return op_lincomb((orc_ctx*)h, (const orc_ct*)a, va, (const orc_ct*)b, vb, target, rescale);
}
ORC_API void orc_automorph(void* h, int t, const uint64_t* in, uint64_t g, uint64_t* out) {
  orc_ctx* c = (orc_ctx*)h;
  automorph_mod(c, in, g, c->mod[t], out);
}
ORC_API uint64_t orc_galois_elt(void* h, int64_t step) { return galois_elt((orc_ctx*)h, step); }

/* ------------------------------------------------------------------------- */
/* Sign polynomials (Sec. 3.2, Eq. 4): f and g are odd, degree 9               */
/* ------------------------------------------------------------------------- */
/* f_4(x) = (315x - 420x^3 + 378x^5 - 180x^7 + 35x^9) / 2^7: the closed form
   sum_{i<=4} binom(2i,i) 4^-i x (1-x^2)^i, whose derivative is c (1-x^2)^4. */
static const double SIGN_F[5] = {315.0 / 128.0, -420.0 / 128.0, 378.0 / 128.0, -180.0 / 128.0, 35.0 / 128.0};
/* g_4 of Cheon-Kim-Kim (ASIACRYPT 2020), odd coefficients of x, x^3, ..., x^9 over 2^10 */
static const double SIGN_G[5] = {5850.0 / 1024.0, -34974.0 / 1024.0, 97015.0 / 1024.0, -113492.0 / 1024.0, 46623.0 / 1024.0};

ORC_API void orc_sign_coeffs(double* f, double* g) {
  memcpy(f, SIGN_F, sizeof(SIGN_F));
  memcpy(g, SIGN_G, sizeof(SIGN_G));
}

/* p(x) = (c1 x + c3 x^3) + x^4 (c5 x + c7 x^3) + x^8 (c9 x): baby steps x^2,
   x^3, x^4, giant step x^8; B and C as constant combinations rescaled once; A
   as a combination that is not rescaled, at the scale of the products;
   x^4 B + x^8 C + A summed as degree-2 ciphertexts and relinearised once.
   Depth 4, five relinearisations.  Output at level l-4 with scale 'target' (up
   to the FP64 rounding of the scale bookkeeping).  c[] = c1, c3, c5, c7, c9,
   times 'gain'. */
/* ct x ct as the textbook evaluator does it (Sec. 2.2): tensor, relinearise
   (hybrid key switch of the s^2 part), then rescale by the top prime */
static orc_ct* op_mul_relin_then_rescale(orc_ctx* c, const orc_ct* a, const orc_ct* b) {
  orc_ct* x = op_mul_relin(c, a, b);
  rescale_inplace(c, x);
  return x;
}

/* The same odd polynomial with the textbook evaluator: every product
   relinearised and then rescaled on its own, every constant combination
   rescaled once:
     x^2 = x x, x^3 = x^2 x, x^4 = x^2 x^2, x^8 = x^4 x^4       (levels l-1 .. l-3)
     A = c1 x + c3 x^3, B = c5 x + c7 x^3, C = c9 x            (level l-3)
     p = x^4 B + x^8 C + A                                      (level l-4)
   Six key switches, depth 4, and the scales of the merged form: the products
   land on (T q_{l-3}) / q_{l-3} and A is taken to that scale exactly. */
static orc_ct* eval_odd9_textbook(orc_ctx* c, const orc_ct* x, const double* coef, double gain, double target) {
  int l = x->level;
  if (l - 4 < c->min_level) die("eval_odd9: not enough levels");
  double k1 = coef[0] * gain, k3 = coef[1] * gain, k5 = coef[2] * gain, k7 = coef[3] * gain, k9 = coef[4] * gain;
  orc_ct* x2 = op_mul_relin_then_rescale(c, x, x);            /* l-1 */
  orc_ct* x3 = op_mul_relin_then_rescale(c, x2, x);           /* l-2 */
  orc_ct* x4 = op_mul_relin_then_rescale(c, x2, x2);          /* l-2 */
  orc_ct* x8 = op_mul_relin_then_rescale(c, x4, x4);          /* l-3 */
  orc_ct* xl2 = ct_copy(c, x, l - 2);
  double q3 = (double)c->mod[l - 3];
  double ta = target * q3;
  double sb = ta / x4->scale;
  double sc = ta / x8->scale;
  orc_ct* B = op_lincomb(c, xl2, k5, x3, k7, sb, 1);          /* l-3 */
  orc_ct* Cc = op_lincomb(c, xl2, k9, NULL, 0.0, sc, 1);      /* l-3 */
  orc_ct* x4l = ct_copy(c, x4, l - 3);
  orc_ct* t = op_mul_relin_then_rescale(c, x4l, B);           /* l-4 */
  orc_ct* u = op_mul_relin_then_rescale(c, x8, Cc);           /* l-4 */
  orc_ct* A3 = op_lincomb(c, xl2, k1, x3, k3, t->scale, 1);   /* l-3 */
  orc_ct* A = ct_copy(c, A3, l - 4);
  orc_ct* tu = op_add(c, t, u, 0);
  orc_ct* p = op_add(c, tu, A, 0);
  ct_free(x2); ct_free(x3); ct_free(x4); ct_free(x8); ct_free(xl2); ct_free(B); ct_free(Cc); ct_free(x4l);
  ct_free(t); ct_free(u); ct_free(A3); ct_free(A); ct_free(tu);
  c->counters[CNT_POLY]++;
  return p;
}

static orc_ct* eval_odd9(orc_ctx* c, const orc_ct* x, const double* coef, double gain, double target) {
  if (c->textbook) return eval_odd9_textbook(c, x, coef, gain, target);
  int l = x->level;
  if (l - 4 < c->min_level) die("eval_odd9: not enough levels");
  double k1 = coef[0] * gain, k3 = coef[1] * gain, k5 = coef[2] * gain, k7 = coef[3] * gain, k9 = coef[4] * gain;
  orc_ct* x2 = op_mul_relin_rescale(c, x, x);                 /* l-1 */
  orc_ct* xl1 = ct_copy(c, x, l - 1);
  orc_ct* x3 = op_mul_relin_rescale(c, x2, xl1);              /* l-2 */
  orc_ct* x4 = op_mul_relin_rescale(c, x2, x2);               /* l-2 */
  orc_ct* x8 = op_mul_relin_rescale(c, x4, x4);               /* l-3 */
  orc_ct* xl2 = ct_copy(c, x, l - 2);
  orc_ct* xl3 = ct_copy(c, x, l - 3);
  orc_ct* x3l3 = ct_copy(c, x3, l - 3);
  double q3 = (double)c->mod[l - 3];
  /* before the last rescale every term carries target * q_{l-3} */
  double ta = target * q3;
  double sb = ta / x4->scale;
  double sc = ta / x8->scale;
  orc_ct* A = op_lincomb(c, xl3, k1, x3l3, k3, ta, 0);        /* l-3, not rescaled */
  orc_ct* B = op_lincomb(c, xl2, k5, x3, k7, sb, 1);          /* l-3 */
  orc_ct* Cc = op_lincomb(c, xl2, k9, NULL, 0.0, sc, 1);      /* l-3 */
  orc_ct* x4l = ct_copy(c, x4, l - 3);
  orc_ct3* t = op_tensor(c, x4l, B);
  orc_ct3* u = op_tensor(c, x8, Cc);
  op_add3_inplace(c, t, u);
  op_add3_ct_inplace(c, t, A);
  orc_ct* p = op_relin_rescale(c, t);                         /* l-4 */
  ct_free(x2); ct_free(xl1); ct_free(x3); ct_free(x4); ct_free(x8); ct_free(xl2); ct_free(xl3); ct_free(x3l3);
  ct_free(A); ct_free(B); ct_free(Cc); ct_free(x4l);
  ct3_free(t); ct3_free(u);
  c->counters[CNT_POLY]++;
  return p;
}

/* 1: the textbook evaluator (every product relinearised, then rescaled; no
   merged relinearise-and-rescale, no lazy relinearisation); 0: the default */
ORC_API void orc_set_textbook(void* h, int on) { ((orc_ctx*)h)->textbook = on ? 1 : 0; }

ORC_API void* orc_eval_odd9(void* h, const void* x, const double* coef, double gain, double target) {
  return eval_odd9((orc_ctx*)h, (const orc_ct*)x, coef, gain, target);
}

/* refresh randomness: the k-th refresh of a chain uses index base + stride * k */
typedef struct {
  uint64_t seed;
  uint64_t next;
  uint64_t stride;
  uint64_t base;
  int span;             /* > 0: only slots [0, span) matter from here on */
} refresher;

static orc_ct* bootstrap(orc_ctx* c, const orc_ct* x);
static orc_ct* bootstrap_sparse(orc_ctx* c, const orc_ct* x);
static orc_ct* maybe_refresh(orc_ctx* c, orc_ct* x, int need, refresher* rf) {
  if (x->level - need >= c->min_level) return x;
  if (c->refresh_level - need < c->min_level) die("modulus chain too short for one unit");
  if (c->boot_mode) {
    int sparse = c->boot_sparse > 0 && rf->span > 0 && rf->span <= c->boot_sparse;
    orc_ct* b = sparse ? bootstrap_sparse(c, x) : bootstrap(c, x);
    ct_free(x);
    return b;
  }
  orc_ct* y = op_refresh(c, x, rf->seed, rf->base + rf->stride * rf->next++);
  ct_free(x);
  return y;
}

/* Sign(x) = f^df(g^dg(x)); the last polynomial is scaled by 'gain' and lands on
   scale 'last_target'; 'last_need' is the number of levels the caller needs
   after the last polynomial beyond its own four. */
static orc_ct* eval_sign(orc_ctx* c, const orc_ct* x_in, double gain, double last_target, int last_extra, refresher* rf,
                         int* last_level_out) {
  double delta = ldexp(1.0, c->log_scale);
  orc_ct* x = ct_copy(c, x_in, x_in->level);
  int total = c->dg + c->df;
  for (int i = 0; i < total; ++i) {
    int last = i == total - 1;
    x = maybe_refresh(c, x, 4 + (last ? last_extra : 0), rf);
    if (last && last_level_out) *last_level_out = x->level - 4;
    const double* coef = i < c->dg ? SIGN_G : SIGN_F;
    orc_ct* y = eval_odd9(c, x, coef, last ? gain : 1.0, last ? last_target : delta);
    ct_free(x);
    x = y;
  }
  c->counters[CNT_SIGN]++;
  return x;
}

/* Max(a, b) = (a+b)/2 + (a-b)/2 * Sign(a-b)   (Eq. 6); a and b share level and scale */
static orc_ct* op_max(orc_ctx* c, const orc_ct* a, const orc_ct* b, refresher* rf) {
  double delta = ldexp(1.0, c->log_scale);
  orc_ct* d = op_add(c, a, b, 1);
  orc_ct* s = op_add(c, a, b, 0);
  int ld = d->level;
  /* the Sign output level is known once the refresh decision for the last
     polynomial is taken; its target scale makes d * Sign/2 land on delta */
  int ls = 0;
  /* first pass: plan the level of the last polynomial without evaluating */
  {
    int lvl = d->level;
    int total = c->dg + c->df;
    for (int i = 0; i < total; ++i) {
      int last = i == total - 1;
      int need = 4 + (last ? 1 : 0);
      if (lvl - need < c->min_level) lvl = c->refresh_level;
      if (lvl - need < c->min_level) die("modulus chain too short for one unit");
      lvl -= 4;
    }
    ls = lvl;
  }
  int lp = ld < ls ? ld : ls;
  double t_sign = delta * (double)c->mod[lp];
  t_sign = t_sign / d->scale;
  int ls_real = -1;
  orc_ct* sg = eval_sign(c, d, 0.5, t_sign, 1, rf, &ls_real);
  if (ls_real != ls) die("op_max: level plan mismatch");
  orc_ct* dl = ct_copy(c, d, lp);
  orc_ct* sgl = ct_copy(c, sg, lp);
  if (c->textbook) {
    /* textbook: d * Sign/2 relinearised, then rescaled; (a+b)/2 as its own
       constant product rescaled to the same level and scale; then added */
    orc_ct* pr = op_mul_relin_then_rescale(c, dl, sgl);
    orc_ct* sl = ct_copy(c, s, lp);
    orc_ct* half = op_lincomb(c, sl, 0.5, NULL, 0.0, pr->scale, 1);
    orc_ct* out = op_add(c, pr, half, 0);
    ct_free(d); ct_free(s); ct_free(sg); ct_free(dl); ct_free(sgl); ct_free(pr); ct_free(sl); ct_free(half);
    c->counters[CNT_MAX]++;
    return out;
  }
  /* d * Sign/2 as a degree-2 ciphertext, (a+b)/2 added at the same scale before
     the one relinearise-and-rescale */
  orc_ct3* prod = op_tensor(c, dl, sgl);
  orc_ct* sl = ct_copy(c, s, lp);
  orc_ct* half = op_lincomb(c, sl, 0.5, NULL, 0.0, prod->scale, 0);
  op_add3_ct_inplace(c, prod, half);
  orc_ct* out = op_relin_rescale(c, prod);
  ct_free(d); ct_free(s); ct_free(sg); ct_free(dl); ct_free(sgl); ct3_free(prod); ct_free(sl); ct_free(half);
  c->counters[CNT_MAX]++;
  return out;
}

static int ilog2_ceil(int v) {
  int r = 0;
  while ((1 << r) < v) ++r;
  return r;
}

/* layout (Eq. 1 with the prompt axis): slot k*C' + c <- logits[k*C + c] */
ORC_API void orc_layout(void* h, const double* logits, int K, int C, double* slots) {
  orc_ctx* c = (orc_ctx*)h;
  int cp = 1 << ilog2_ceil(C);
  for (int j = 0; j < c->n / 2; ++j) slots[j] = 0.0;
  for (int k = 0; k < K; ++k)
    for (int cc = 0; cc < C; ++cc) slots[k * cp + cc] = logits[k * C + cc];
}

ORC_API void* orc_encrypt_logits(void* h, const double* logits, int K, int C, uint64_t seed) {
  orc_ctx* c = (orc_ctx*)h;
  int cp = 1 << ilog2_ceil(C), kp = 1 << ilog2_ceil(K);
  if (kp * cp > c->n / 2) die("K' * C' exceeds the slot count");
  double* slots = (double*)xcalloc(c->n / 2, sizeof(double));
  orc_layout(h, logits, K, C, slots);
  int64_t* m = (int64_t*)xcalloc(c->n, 8);
  encode_real(c, slots, kp * cp, ldexp(1.0, c->log_scale), m);
  void* x = orc_encrypt(h, m, ldexp(1.0, c->log_scale), seed);
  free(slots);
  free(m);
  return x;
}

/* Packed layout (Sec. 3.2 packs N/(2n) Argmax inputs in one ciphertext): n_b
   queries, query b in the block of slots [b*bsz, (b+1)*bsz) at slot
   b*bsz + k*C' + c, with K', C' the largest padded shape of the group and
   bsz = max(K'C', 2C'), so that the prompt sum, the duplication and QuickMax
   of every block stay inside it. */
static void packed_shape(int n_b, const int* K, const int* C, int* kp, int* cp, int* bsz) {
  int lk = 0, lc = 0;
  for (int b = 0; b < n_b; ++b) {
    if (ilog2_ceil(K[b]) > lk) lk = ilog2_ceil(K[b]);
    if (ilog2_ceil(C[b]) > lc) lc = ilog2_ceil(C[b]);
  }
  *kp = 1 << lk;
  *cp = 1 << lc;
  *bsz = *kp * *cp > 2 * *cp ? *kp * *cp : 2 * *cp;
}

/* out3 = {K', C', block size}; returns the number of blocks a ciphertext holds */
ORC_API int orc_packed_shape(void* h, int n_b, const int* K, const int* C, int* out3) {
  orc_ctx* c = (orc_ctx*)h;
  packed_shape(n_b, K, C, &out3[0], &out3[1], &out3[2]);
  return (c->n / 2) / out3[2];
}

/* logits: the queries' K_b x C_b blocks concatenated */
ORC_API void orc_layout_packed(void* h, int n_b, const double* logits, const int* K, const int* C, double* slots) {
  orc_ctx* c = (orc_ctx*)h;
  int kp, cp, bsz;
  packed_shape(n_b, K, C, &kp, &cp, &bsz);
  if ((int64_t)n_b * bsz > c->n / 2) die("packed queries exceed the slot count");
  for (int j = 0; j < c->n / 2; ++j) slots[j] = 0.0;
  const double* y = logits;
  for (int b = 0; b < n_b; ++b) {
    for (int k = 0; k < K[b]; ++k)
      for (int cc = 0; cc < C[b]; ++cc) slots[b * bsz + k * cp + cc] = y[k * C[b] + cc];
    y += K[b] * C[b];
  }
}

ORC_API void* orc_encrypt_packed(void* h, int n_b, const double* logits, const int* K, const int* C, uint64_t seed) {
  orc_ctx* c = (orc_ctx*)h;
  double* slots = (double*)xcalloc(c->n / 2, sizeof(double));
  orc_layout_packed(h, n_b, logits, K, C, slots);
  int64_t* m = (int64_t*)xcalloc(c->n, 8);
  encode_real(c, slots, c->n / 2, ldexp(1.0, c->log_scale), m);
  void* x = orc_encrypt(h, m, ldexp(1.0, c->log_scale), seed);
  free(slots);
  free(m);
  return x;
}

/* The encrypted Argmax (Algorithm 1) over the prompt-summed logits.
   y[k*C'+c] holds the k-th prompt's score for class c.  Steps:
     prompt sum   y <- y + RotL(y, C' 2^i), i < log K'   (sum by doubling, Sec. 3.2)
     normalise    y <- mask_[0,C) * (y - D_min) / (D_max - D_min)   (Eq. 5)
     line 2       y <- y + RotR(y, C')
     line 3       y_max <- QuickMax(y): y <- Max(RotL(y, 2^i), y), i < log C'
     line 4       y <- y - y_max
     lines 5-6    z <- Sign(y) + 1                                   (Eq. 2) */
static orc_ct* eval_argmax_core(orc_ctx* c, const orc_ct* ct_in, int lk, int lc, int packed, int n_b, int bsz,
                                const int* C, const double* d_min, const double* d_max, uint64_t refresh_seed) {
  double delta = ldexp(1.0, c->log_scale);
  int cp = 1 << lc;
  int slots = c->n / 2;
  /* after Eq. 5 only slots [0, 2C') of a single query's ciphertext are read
     again (the duplicate of line 2 and the QuickMax windows stay inside) */
  refresher rf = {refresh_seed, 0, 1, 0, packed ? 0 : 2 * cp};
  orc_ct* y = ct_copy(c, ct_in, ct_in->level);
  for (int i = 0; i < lk; ++i) {
    orc_ct* r = op_rotate(c, y, (int64_t)cp << i);
    orc_ct* s = op_add(c, y, r, 0);
    ct_free(r); ct_free(y);
    y = s;
  }
  /* normalise; y must keep one level for the mask product */
  y = maybe_refresh(c, y, 1, &rf);
  orc_ct* yn;
  if (!packed) {
    op_add_const_inplace(c, y, -d_min[0]);
    double* mask = (double*)xcalloc(cp, sizeof(double));
    double inv_range = 1.0 / (d_max[0] - d_min[0]);
    for (int j = 0; j < C[0]; ++j) mask[j] = inv_range;
    yn = op_mul_plain(c, y, mask, cp, delta);
    free(mask);
  } else {
    /* per block: -D_min on its classes, then the mask 1/(D_max - D_min) there */
    int used = n_b * bsz;
    double* shift = (double*)xcalloc(used, sizeof(double));
    double* mask = (double*)xcalloc(used, sizeof(double));
    for (int b = 0; b < n_b; ++b) {
      double inv_range = 1.0 / (d_max[b] - d_min[b]);
      for (int j = 0; j < C[b]; ++j) {
        shift[b * bsz + j] = -d_min[b];
        mask[b * bsz + j] = inv_range;
      }
    }
    orc_ct* y1 = op_add_plain(c, y, shift, used);
    yn = op_mul_plain(c, y1, mask, used, delta);
    ct_free(y1);
    free(shift);
    free(mask);
  }
  ct_free(y);
  /* line 2: duplicate */
  orc_ct* r = op_rotate(c, yn, (int64_t)slots - cp);
  orc_ct* ydup = op_add(c, yn, r, 0);
  ct_free(r); ct_free(yn);
  /* line 3: QuickMax */
  orc_ct* ym = ct_copy(c, ydup, ydup->level);
  for (int i = 0; i < lc; ++i) {
    ym = maybe_refresh(c, ym, 1, &rf);
    orc_ct* rot = op_rotate(c, ym, (int64_t)1 << i);
    orc_ct* mx = op_max(c, rot, ym, &rf);
    ct_free(rot); ct_free(ym);
    ym = mx;
  }
  /* line 4 */
  orc_ct* d = op_add(c, ydup, ym, 1);
  ct_free(ydup); ct_free(ym);
  /* lines 5-6 */
  orc_ct* z = eval_sign(c, d, 1.0, delta, 0, &rf, NULL);
  ct_free(d);
  op_add_const_inplace(c, z, 1.0);
  return z;
}

ORC_API void* orc_eval_argmax(void* h, const void* ct_in, int K, int C, double d_min, double d_max, uint64_t refresh_seed) {
  return eval_argmax_core((orc_ctx*)h, (const orc_ct*)ct_in, ilog2_ceil(K), ilog2_ceil(C), 0, 1, 0, &C, &d_min,
                          &d_max, refresh_seed);
}

/* The comparison path the paper measures against (Phoenix, Sec. 3.2): after
   the same prompt sum and Eq. 5, every class is compared with each of the
   other C-1 classes,
     s = sum_{i=1}^{C-1} Sign(y - RotL(y, i))     (y duplicated at offset C),
   so the largest class reaches s = C-1 and every other s <= C-3; then
     z = (Sign((s - (C-2)) / (2C-3)) + 1) / 2
   turns s into the one-hot vector (the paper leaves this last linear map to
   the Phoenix paper; this is the reading).  C Signs and C rotations.  The
   k-th refresh of comparison i (i = 0 for the prefix and the final Sign)
   uses refresh index k * 512 + i. */
#define PHOENIX_STRIDE 512
ORC_API void* orc_eval_argmax_phoenix(void* h, const void* ct_in, int K, int C, double d_min, double d_max,
                                      uint64_t refresh_seed) {
  orc_ctx* c = (orc_ctx*)h;
  if (C < 2 || C >= PHOENIX_STRIDE) die("phoenix path: need 2 <= C < 512");
  double delta = ldexp(1.0, c->log_scale);
  int lk = ilog2_ceil(K), cp = 1 << ilog2_ceil(C);
  int slots = c->n / 2;
  if ((int64_t)(1 << lk) * cp > slots || 2 * C > slots) die("phoenix path: shape exceeds the slot count");
  refresher rf0 = {refresh_seed, 0, PHOENIX_STRIDE, 0, 0};
  orc_ct* y = ct_copy(c, (const orc_ct*)ct_in, ((const orc_ct*)ct_in)->level);
  for (int i = 0; i < lk; ++i) {
    orc_ct* r = op_rotate(c, y, (int64_t)cp << i);
    orc_ct* t = op_add(c, y, r, 0);
    ct_free(r); ct_free(y);
    y = t;
  }
  y = maybe_refresh(c, y, 1, &rf0);
  op_add_const_inplace(c, y, -d_min);
  double* mask = (double*)xcalloc(cp, sizeof(double));
  double inv_range = 1.0 / (d_max - d_min);
  for (int j = 0; j < C; ++j) mask[j] = inv_range;
  orc_ct* yn = op_mul_plain(c, y, mask, cp, delta);
  free(mask);
  ct_free(y);
  orc_ct* r = op_rotate(c, yn, (int64_t)slots - C);
  orc_ct* yd = op_add(c, yn, r, 0);
  ct_free(r); ct_free(yn);
  orc_ct* s = NULL;
  for (int i = 1; i < C; ++i) {
    refresher rfi = {refresh_seed, 0, PHOENIX_STRIDE, (uint64_t)i, 0};
    orc_ct* ri = op_rotate(c, yd, i);
    orc_ct* di = op_add(c, yd, ri, 1);
    orc_ct* si = eval_sign(c, di, 1.0, delta, 0, &rfi, NULL);
    ct_free(ri); ct_free(di);
    if (!s) {
      s = si;
    } else {
      orc_ct* t = op_add(c, s, si, 0);
      ct_free(s); ct_free(si);
      s = t;
    }
  }
  ct_free(yd);
  /* x = (s - (C - 2)) / (2C - 3), one level for the constant product */
  s = maybe_refresh(c, s, 1, &rf0);
  op_add_const_inplace(c, s, -(double)(C - 2));
  orc_ct* x = op_mul_const(c, s, 1.0 / (double)(2 * C - 3), delta);
  ct_free(s);
  orc_ct* z = eval_sign(c, x, 0.5, delta, 0, &rf0, NULL);
  ct_free(x);
  op_add_const_inplace(c, z, 0.5);
  return z;
}

/* Algorithm 1 on every block of a packed ciphertext at once (same steps, with
   K', C' of the group; Eq. 5 with each block's own bounds and classes) */
ORC_API void* orc_eval_argmax_packed(void* h, const void* ct_in, int n_b, const int* K, const int* C,
                                     const double* d_min, const double* d_max, uint64_t refresh_seed) {
  orc_ctx* c = (orc_ctx*)h;
  int kp, cp, bsz;
  packed_shape(n_b, K, C, &kp, &cp, &bsz);
  if ((int64_t)n_b * bsz > c->n / 2) die("packed queries exceed the slot count");
  return eval_argmax_core(c, (const orc_ct*)ct_in, ilog2_ceil(kp), ilog2_ceil(cp), 1, n_b, bsz, C, d_min, d_max,
                          refresh_seed);
}

/* ========================================================================= */
/* bootstrapping                                                              */
/* ========================================================================= */
/* The paper refreshes by bootstrapping (Sec. 2.2; Sec. 4.1: K = 14 levels of
   L = 35) and cites full-RNS CKKS bootstrapping without giving its steps.
   This is the standard pipeline, step by step:
     scale-down   the level-1 input times one constant lands on level 0 with
                  scale T_b = q_0 2^-ratio, so |m| <= q_0 2^-ratio for |z| <= 1;
     ModRaise     centred lift of the level-0 residues to every chain prime:
                  the result decrypts to t = m + q_0 I with I small (sparse
                  secret) and is declared at scale q_0, so its slots hold
                  U (t_lo + i t_hi) / q_0 with U_jk = zeta^(5^j k), j, k < N/2;
     CoeffToSlot  U^-1 = P F_1^-1 ... F_L^-1, P the bit reversal, F_m the
                  radix-2 butterfly stages of the special FFT (Cheon, Han,
                  Kim, Kim, Song, SAC 2018), merged into groups of one level,
                  each evaluated with baby-step giant-step diagonals; the
                  conjugation then splits real and imaginary parts;
     EvalMod      x = t / q_0 mod 1 through cos(2 pi (x - 1/4) / 2^r) as a
                  Chebyshev interpolant on [-(K+1), K+1] and r double angles
                  cos 2a = 2 cos^2 a - 1 (Han, Ki, CT-RSA 2020), which leaves
                  sin(2 pi x) ~ 2 pi m / q_0;
     SlotToCoeff  F_L ... F_1 with 2^ratio / (2 pi) folded in, back to z at
                  scale Delta.
   Slot vectors of the linear transforms are computed in binary128 and
   rounded to binary64 before encoding. */

typedef struct { __float128 re, im; } cq;
static inline cq cq_mul(cq a, cq b) { cq r = {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re}; return r; }

/* zeta^t = exp(i pi t / N) from the binary128 cosine table */
static cq zeta_pow(orc_ctx* c, uint64_t t) {
  uint64_t m2n = 2ull * (uint64_t)c->n;
  t %= m2n;
  cq r = {c->cos_tab[t], c->cos_tab[(t + 3ull * (uint64_t)c->n / 2) % m2n]};
  return r;
}

/* m_k = round(scale * 2/N * Re sum_j z_j zeta^(-5^j k)) for complex slot values */
static void encode_complex(orc_ctx* c, const double* re, const double* im, int nslots, double scale, int64_t* m) {
  int n = c->n;
  uint64_t m2n = 2ull * (uint64_t)n;
  __float128 f = (__float128)scale * 2 / (__float128)n;
  for (int k = 0; k < n; ++k) {
    __float128 acc = 0;
    for (int j = 0; j < nslots; ++j) {
      if (re[j] == 0.0 && im[j] == 0.0) continue;
      uint64_t t = (c->rot_group[j] * (uint64_t)k) % m2n;
      acc += (__float128)re[j] * c->cos_tab[t] + (__float128)im[j] * c->cos_tab[(t + 3ull * (uint64_t)n / 2) % m2n];
    }
    m[k] = round_half_away_q(f * acc);
  }
}
ORC_API void orc_encode_complex(void* h, const double* re, const double* im, int nslots, double scale, int64_t* m) {
  encode_complex((orc_ctx*)h, re, im, nslots, scale, m);
}

/* a matrix on the S slots as generalised diagonals: out[p] = sum_d D[d][p] in[(p+d) mod S] */
typedef struct { int S; cq** d; } diagmat;
static diagmat dm_new(int S) { diagmat m = {S, (cq**)xcalloc(S, sizeof(cq*))}; return m; }
static void dm_free(diagmat* m) {
  for (int i = 0; i < m->S; ++i) free(m->d[i]);
  free(m->d);
}
static cq* dm_at(diagmat* m, int off) {
  if (!m->d[off]) m->d[off] = (cq*)xcalloc(m->S, sizeof(cq));
  return m->d[off];
}
/* one radix-2 stage on blocks of m slots, D_m[j] = zeta^((N/2m) 5^j):
   forward  out[r] = in[r] + D[r] in[r+h],  out[r+h] = in[r] - D[r] in[r+h]   (h = m/2)
   inverse  out[r] = (in[r] + in[r+h]) / 2, out[r+h] = conj(D[r]) (in[r] - in[r+h]) / 2
   as a map on S = ns slots.  The stages of the n-slot special FFT (root
   zeta^(N/2n) of order 4n) have the same twiddles zeta^((N/2m) 5^j). */
static diagmat dm_stage(orc_ctx* c, int m, int inverse, int ns) {
  int S = ns, h = m / 2;
  diagmat A = dm_new(S);
  for (int p = 0; p < S; ++p) {
    int r = p % m;
    int j = r < h ? r : r - h;
    cq D = zeta_pow(c, (uint64_t)(c->n / 2 / m) * c->rot_group[j]);
    if (!inverse) {
      if (r < h) {
        dm_at(&A, 0)[p] = (cq){1, 0};
        dm_at(&A, h % S)[p] = D;
      } else {
        dm_at(&A, 0)[p] = (cq){-D.re, -D.im};
        dm_at(&A, (S - h) % S)[p] = (cq){1, 0};
      }
    } else {
      if (r < h) {
        dm_at(&A, 0)[p] = (cq){0.5Q, 0};
        dm_at(&A, h % S)[p] = (cq){0.5Q, 0};
      } else {
        cq Dc = {D.re / 2, -D.im / 2};
        dm_at(&A, (S - h) % S)[p] = Dc;
        dm_at(&A, 0)[p] = (cq){-Dc.re, -Dc.im};
      }
    }
  }
  return A;
}
/* A B (B applied first): (AB)[d1+d2][p] += A[d1][p] B[d2][p+d1] */
static diagmat dm_mul(const diagmat* A, const diagmat* B) {
  int S = A->S;
  diagmat R = dm_new(S);
  for (int d1 = 0; d1 < S; ++d1) {
    if (!A->d[d1]) continue;
    for (int d2 = 0; d2 < S; ++d2) {
      if (!B->d[d2]) continue;
      cq* out = dm_at(&R, (d1 + d2) % S);
      for (int p = 0; p < S; ++p) {
        cq t = cq_mul(A->d[d1][p], B->d[d2][(p + d1) % S]);
        out[p].re += t.re;
        out[p].im += t.im;
      }
    }
  }
  return R;
}

/* the groups of stages: L = log2 S stages split into 'groups' runs, the
   larger runs first; CoeffToSlot applies m = S, S/2, ..., 2, SlotToCoeff
   m = 2, 4, ..., S.  Group g covers stages [first, first + len) of that order. */
static int boot_group_len(int L, int groups, int g) { return L / groups + (g < L % groups ? 1 : 0); }
static int boot_stage_m(int L, int inverse, int idx) { return inverse ? 1 << (L - idx) : 1 << (idx + 1); }

/* baby-step size for a group of g stages: 2^ceil((g+1)/2), at most E */
static int boot_n1(int g, int E) {
  int n1 = 1 << ((g + 2) / 2);
  return n1 > E ? E : n1;
}
static int64_t floor_div(int64_t a, int64_t b) { return a >= 0 ? a / b : -((-a + b - 1) / b); }

typedef struct {
  int inverse, level;           /* level of the input ciphertext */
  int ns;                       /* slots of the transform: N/2, or n (sparse) */
  int delta, n1, E;             /* offsets are multiples of delta; E = ns / delta */
  diagmat M;
} boot_group;

/* group g of 'groups' over an ns-slot transform (ns = N/2: the full one) */
static boot_group boot_make_group_ns(orc_ctx* c, int inverse, int g, int level, int ns, int groups) {
  int S = ns, L = 0;
  while ((1 << L) < S) ++L;
  int first = 0;
  for (int i = 0; i < g; ++i) first += boot_group_len(L, groups, i);
  int len = boot_group_len(L, groups, g);
  boot_group G;
  G.inverse = inverse;
  G.level = level;
  G.ns = ns;
  int mmin = S;
  diagmat M = dm_stage(c, boot_stage_m(L, inverse, first), inverse, ns);
  if (boot_stage_m(L, inverse, first) < mmin) mmin = boot_stage_m(L, inverse, first);
  for (int i = 1; i < len; ++i) {
    int m = boot_stage_m(L, inverse, first + i);
    if (m < mmin) mmin = m;
    diagmat St = dm_stage(c, m, inverse, ns);
    diagmat R = dm_mul(&St, &M);
    dm_free(&St);
    dm_free(&M);
    M = R;
  }
  /* constants folded into the first group applied; a sparse CoeffToSlot
     also undoes the factor N/(2n) of the trace before it */
  if (g == 0) {
    __float128 k = inverse ? 1.0Q / (2.0Q * (__float128)(c->boot_K + 1))
                           : ldexpq(1.0Q, c->boot_ratio) / (2.0Q * M_PIq);
    if (inverse) k = k * (__float128)ns / (__float128)(c->n / 2);
    for (int d = 0; d < S; ++d)
      if (M.d[d])
        for (int p = 0; p < S; ++p) { M.d[d][p].re *= k; M.d[d][p].im *= k; }
  }
  G.M = M;
  G.delta = mmin / 2;
  G.E = S / G.delta;
  G.n1 = boot_n1(len, G.E);
  return G;
}
static boot_group boot_make_group(orc_ctx* c, int inverse, int g, int level) {
  return boot_make_group_ns(c, inverse, g, level, c->n / 2, c->boot_groups);
}

/* centred multiple e of delta for slot offset d: e in [-E/2, E/2) */
static int64_t boot_e(const boot_group* G, int d) {
  int64_t e = d / G->delta;
  if (e >= G->E / 2) e -= G->E;
  return e;
}

/* one group = one level: out = sum_G Rot( sum_b pt_{G,b} * Rot(x, delta b), delta n1 G ),
   pt_{G,b} = the diagonal of e = n1 G + b rotated right by delta n1 G, encoded at
   p = T q_l / s; the sum is rescaled once and carries scale T */
static orc_ct* boot_apply_group(orc_ctx* c, const boot_group* G, int g, const orc_ct* x, double target) {
  int S = G->ns, SF = c->n / 2, n = c->n, l = x->level;
  if (l != G->level) die("boot group: level mismatch");
  double ql = (double)c->mod[l];
  double pscale = target * ql;
  pscale = pscale / x->scale;
  int64_t gmin = floor_div(-(int64_t)G->E / 2, G->n1), gmax = floor_div((int64_t)G->E / 2 - 1, G->n1);
  int n_g = (int)(gmax - gmin + 1);
  /* which baby steps are used */
  int* used = (int*)xcalloc(G->n1, sizeof(int));
  for (int d = 0; d < S; ++d) {
    if (!G->M.d[d]) continue;
    int64_t e = boot_e(G, d);
    used[e - G->n1 * floor_div(e, G->n1)] = 1;
  }
  /* the baby steps share one ModUp (hoisted rotations) */
  orc_ct** xb = (orc_ct**)xcalloc(G->n1, sizeof(orc_ct*));
  int64_t* bst = (int64_t*)xcalloc(G->n1, sizeof(int64_t));
  int* bidx = (int*)xcalloc(G->n1, sizeof(int));
  orc_ct** bout = (orc_ct**)xcalloc(G->n1, sizeof(orc_ct*));
  int nb = 0;
  for (int b = 0; b < G->n1; ++b) {
    if (!used[b]) continue;
    if (b == 0) {
      xb[0] = ct_copy(c, x, l);
    } else {
      bst[nb] = (int64_t)G->delta * b;
      bidx[nb++] = b;
    }
  }
  op_rotate_hoisted(c, x, bst, nb, bout);
  for (int i = 0; i < nb; ++i) xb[bidx[i]] = bout[i];
  free(bst);
  free(bidx);
  free(bout);
  orc_ct* out = NULL;
  /* the encoded diagonals are kept per (direction, group, plaintext scale) */
  struct boot_pt* cache = c->boot_cache;
  while (cache && !(cache->inverse == G->inverse && cache->g == g && cache->ns == S && cache->pscale == pscale))
    cache = cache->next;
  if (!cache) {
    cache = (struct boot_pt*)xcalloc(1, sizeof(struct boot_pt));
    cache->inverse = G->inverse;
    cache->g = g;
    cache->ns = S;
    cache->pscale = pscale;
    cache->m = (int64_t**)xcalloc(SF, sizeof(int64_t*));
    cache->next = c->boot_cache;
    c->boot_cache = cache;
  }
  double* re = (double*)xcalloc(SF, sizeof(double));
  double* im = (double*)xcalloc(SF, sizeof(double));
  int64_t* m = (int64_t*)xcalloc(n, 8);
  uint64_t* mp = (uint64_t*)xcalloc(n, 8);
  uint64_t* tmp = (uint64_t*)xcalloc(n, 8);
  for (int gi = 0; gi < n_g; ++gi) {
    int64_t gg = gmin + gi;
    orc_ct* inner = NULL;
    for (int d = 0; d < S; ++d) {
      if (!G->M.d[d]) continue;
      int64_t e = boot_e(G, d);
      if (floor_div(e, G->n1) != gg) continue;
      int b = (int)(e - G->n1 * gg);
      if (!cache->m[d]) {
        /* the diagonal repeats with period ns over the N/2 slots */
        int64_t shift = ((G->delta * G->n1 * gg) % S + S) % S;
        for (int p = 0; p < SF; ++p) {
          cq v = G->M.d[d][((int64_t)(p % S) - shift + S) % S];
          re[p] = (double)v.re;
          im[p] = (double)v.im;
        }
        cache->m[d] = (int64_t*)xcalloc(n, 8);
        encode_complex(c, re, im, SF, pscale, cache->m[d]);
      }
      memcpy(m, cache->m[d], 8 * (size_t)n);
      if (!inner) inner = ct_new(c, l, x->scale * pscale);
      for (int t = 0; t <= l; ++t) {
        uint64_t q = c->mod[t];
        poly_from_small(c, m, t, mp);
        for (int pp = 0; pp < 2; ++pp) {
          ring_mul(c, t, LIMB(xb[b], pp, t, n), mp, tmp);
          uint64_t* w = LIMB(inner, pp, t, n);
          for (int i = 0; i < n; ++i) w[i] = madd(w[i], tmp[i], q);
        }
      }
    }
    if (!inner) continue;
    orc_ct* r = gg == 0 ? inner : op_rotate(c, inner, (int64_t)G->delta * G->n1 * gg);
    if (r != inner) ct_free(inner);
    if (!out) {
      out = r;
    } else {
      orc_ct* t = op_add(c, out, r, 0);
      ct_free(out);
      ct_free(r);
      out = t;
    }
  }
  for (int b = 0; b < G->n1; ++b) ct_free(xb[b]);
  free(xb); free(used); free(re); free(im); free(m); free(mp); free(tmp);
  rescale_inplace(c, out);
  out->scale = target;
  return out;
}

/* baby and giant steps of every group of an ns-slot transform (S-slot steps) */
static int boot_transform_steps(orc_ctx* c, int ns, int groups, int64_t* st, int k) {
  int S = c->n / 2, L = 0;
  while ((1 << L) < ns) ++L;
  for (int inv = 0; inv < 2; ++inv)
    for (int g = 0; g < groups; ++g) {
      int first = 0;
      for (int i = 0; i < g; ++i) first += boot_group_len(L, groups, i);
      int len = boot_group_len(L, groups, g);
      int mmin = ns;
      for (int i = 0; i < len; ++i) {
        int mm = boot_stage_m(L, inv, first + i);
        if (mm < mmin) mmin = mm;
      }
      int delta = mmin / 2, E = ns / delta, n1 = boot_n1(len, E);
      for (int b = 1; b < n1; ++b) st[k++] = (int64_t)delta * b % S;
      /* the group's offsets are delta e, |e| <= 2^len - 1, centred in [-E/2, E/2) */
      int64_t span = ((int64_t)1 << len) - 1;
      int64_t elo = span < E / 2 ? -span : -(int64_t)E / 2, ehi = span < E / 2 - 1 ? span : (int64_t)E / 2 - 1;
      int64_t gmin = floor_div(elo, n1), gmax = floor_div(ehi, n1);
      for (int64_t gg = gmin; gg <= gmax; ++gg)
        if (gg) st[k++] = (((int64_t)delta * n1 * gg) % S + S) % S;
    }
  return k;
}

static boot_group boot_make_group_sparse(orc_ctx* c, int inverse, int g, int level);

/* rotation steps one bootstrap uses (CONJ_STEP for the conjugation), and the
   sparse-slot bootstrap's when it is set */
static int boot_steps(orc_ctx* c, int64_t* out, int cap) {
  int S = c->n / 2, k = 0;
  int64_t* st = (int64_t*)xcalloc(8192, sizeof(int64_t));
  k = boot_transform_steps(c, S, c->boot_groups, st, k);
  if (c->boot_sparse > 0) {
    /* the sparse groups' baby steps and the giant steps of the offsets present */
    for (int inv = 0; inv < 2; ++inv)
      for (int g = 0; g < c->boot_groups; ++g) {
        boot_group G = boot_make_group_sparse(c, inv, g, 0);
        for (int b = 1; b < G.n1; ++b) st[k++] = (int64_t)G.delta * b % S;
        for (int d = 0; d < G.ns; ++d) {
          if (!G.M.d[d]) continue;
          int64_t gg = floor_div(boot_e(&G, d), G.n1);
          if (gg) st[k++] = (((int64_t)G.delta * G.n1 * gg) % S + S) % S;
        }
        dm_free(&G.M);
      }
    for (int64_t r = c->boot_sparse; r < S; r *= 2) st[k++] = r;
    st[k++] = S - c->boot_sparse;
  }
  /* sort, unique, drop multiples of S */
  for (int i = 1; i < k; ++i)
    for (int j = i; j > 0 && st[j - 1] > st[j]; --j) { int64_t t = st[j]; st[j] = st[j - 1]; st[j - 1] = t; }
  int u = 0;
  for (int i = 0; i < k; ++i)
    if (st[i] % S != 0 && (u == 0 || st[u - 1] != st[i])) st[u++] = st[i];
  st[u++] = CONJ_STEP;
  for (int i = 0; i < u && i < cap; ++i) out[i] = st[i];
  free(st);
  return u;
}
ORC_API int orc_boot_steps(void* h, int64_t* out, int cap) { return boot_steps((orc_ctx*)h, out, cap); }

/* Chebyshev interpolant of f(u) = cos(2 pi ((K+1) u - 1/4) / 2^r) on [-1, 1] at
   the deg+1 Chebyshev nodes, in binary128:
   c_j = (2 - [j = 0]) / n sum_k f(cos th_k) cos(j th_k), th_k = pi (k + 1/2) / n */
static void boot_cheb_coeffs(int K, int r, int deg, double* out) {
  int n = deg + 1;
  for (int j = 0; j <= deg; ++j) {
    __float128 acc = 0;
    for (int k = 0; k < n; ++k) {
      __float128 th = M_PIq * ((__float128)k + 0.5Q) / (__float128)n;
      __float128 u = cosq(th);
      __float128 f = cosq(2.0Q * M_PIq * ((__float128)(K + 1) * u - 0.25Q) / ldexpq(1.0Q, r));
      acc += f * cosq((__float128)j * th);
    }
    acc = acc * 2.0Q / (__float128)n;
    if (j == 0) acc /= 2;
    out[j] = (double)acc;
  }
}
ORC_API void orc_boot_cheb(void* h, double* out) {
  orc_ctx* c = (orc_ctx*)h;
  memcpy(out, c->boot_cheb, sizeof(double) * (size_t)(c->boot_deg + 1));
}

/* multiply by +-X^(N/2): every slot times +-i (5^j = 1 mod 4) */
static orc_ct* op_mul_monomial_half(orc_ctx* c, const orc_ct* a, int neg) {
  int n = c->n, h = n / 2;
  orc_ct* x = ct_new(c, a->level, a->scale);
  for (int p = 0; p < 2; ++p)
    for (int t = 0; t <= a->level; ++t) {
      uint64_t q = c->mod[t];
      const uint64_t* u = LIMB(a, p, t, n);
      uint64_t* w = LIMB(x, p, t, n);
      for (int i = 0; i < n; ++i) {
        int j = i + h;
        uint64_t v = j < n ? u[i] : mneg(u[i], q);
        if (neg) v = mneg(v, q);
        w[j < n ? j : j - n] = v;
      }
    }
  return x;
}

/* level-0 residues, centred, lifted to every chain prime; declared at scale q_0 */
static orc_ct* mod_raise(orc_ctx* c, const orc_ct* a) {
  if (a->level != 0) die("mod_raise: input must be at level 0");
  int n = c->n, top = c->n_q - 1;
  uint64_t q0 = c->mod[0];
  orc_ct* x = ct_new(c, top, (double)q0);
  for (int p = 0; p < 2; ++p)
    for (int i = 0; i < n; ++i) {
      uint64_t v = a->c[p][i];
      i128 w = v > q0 / 2 ? (i128)v - (i128)q0 : (i128)v;
      for (int t = 0; t <= top; ++t) LIMB(x, p, t, n)[i] = from_i128(w, c->mod[t]);
    }
  return x;
}

/* relinearise a degree-2 ciphertext without rescaling: (d0, d1) + KS(d2) */
static orc_ct* op_relin3(orc_ctx* c, const orc_ct3* x) {
  int l = x->level, n = c->n;
  orc_key* rk = find_key(c, 0);
  if (!rk) die("no relinearisation key");
  orc_ct* out = ct_new(c, l, x->scale);
  uint64_t* u0 = (uint64_t*)xcalloc((size_t)(l + 1) * n, 8);
  uint64_t* u1 = (uint64_t*)xcalloc((size_t)(l + 1) * n, 8);
  key_switch(c, x->c[2], l, rk, u0, u1);
  for (int t = 0; t <= l; ++t) {
    uint64_t q = c->mod[t];
    for (int i = 0; i < n; ++i) {
      size_t o = (size_t)t * n + i;
      out->c[0][o] = madd(x->c[0][o], u0[o], q);
      out->c[1][o] = madd(x->c[1][o], u1[o], q);
    }
  }
  free(u0);
  free(u1);
  c->counters[CNT_RELIN]++;
  return out;
}

/* x^2 relinearised, then rescaled by exact rounding (one level) */
static orc_ct* op_square_exact(orc_ctx* c, const orc_ct* a) {
  orc_ct* p = op_mul_relin(c, a, a);
  rescale_inplace(c, p);
  return p;
}

/* x * 2 (an exact integer product: the constant is 2 at the same scale) */
static orc_ct* op_double(orc_ctx* c, const orc_ct* a) { return op_lincomb(c, a, 2.0, NULL, 0.0, a->scale, 0); }

/* EvalMod on u = x / (K+1) (Han, Ki 2020): p(u) = sum_j c_j T_j(u), the
   Chebyshev interpolant of cos(2 pi ((K+1) u - 1/4) / 2^r), then r double
   angles y <- 2 y^2 - 1.

   p is evaluated baby-step giant-step in the Chebyshev basis: baby steps
   T_1 .. T_(B-1) (B = 2^ceil(k/2) for degree 2^k - 1), giant steps T_B, T_2B,
   .., T_(2^(k-1)); a polynomial of degree < 2h (h a giant) splits by Chebyshev
   division, T_(h+j) = 2 T_h T_j - T_(h-j), into p = r + T_h q with
     q_0 = c_h, q_j = 2 c_(h+j),   r_0 = c_0, r_j = c_j - c_(2h-j)   (0 < j < h),
   recursively, down to combinations of the baby steps.  Each split costs one
   product: (2^m1 - 2) + (k - m1) + (2^(k-m1) - 1) products in all (11 for
   degree 31, against 30 for the whole basis), depth k + 1.  Scales: every node
   lands exactly on the scale its parent needs (its q child's target is
   T q_l / s_h); an r child that is a combination of baby steps is added,
   unrescaled, at the product's scale before relinearising, its constant
   after.  The basis products:
     T_2a    = 2 T_a^2 - 1          (square, doubled, constant subtracted)
     T_(a+b) = 2 T_a T_b - T_(a-b)  (b < a, a the largest power of two below
                                     a+b; (2 T_a) (x) T_b with -T_(a-b) added
                                     before relinearising).
   Every product here is relinearised and then rescaled by exact rounding: the
   merged relinearise-and-rescale rounds through an approximate conversion
   whose error (up to (alpha + 1) / 2 per coefficient) the double angles would
   amplify. */

/* sum_{0 < j < n} cf[j] T_j, every T_j lowered to level lv, at scale 'scale'
   (not rescaled) */
static orc_ct* cheb_combination(orc_ctx* c, orc_ct** T, const double* cf, int n, int lv, double scale) {
  orc_ct* acc = NULL;
  for (int j = 1; j < n; ++j) {
    orc_ct* a1 = ct_copy(c, T[j], lv);
    orc_ct* t = op_lincomb(c, a1, cf[j], NULL, 0.0, scale, 0);
    ct_free(a1);
    if (!acc) {
      acc = t;
    } else {
      orc_ct* s2 = op_add(c, acc, t, 0);
      ct_free(acc);
      ct_free(t);
      acc = s2;
    }
  }
  return acc;
}

/* sum_{j < 2^m} cf[j] T_j with scale exactly 'target'; baby steps below B,
   their deepest level lb; a node of 2^m terms ends at level lb - 1 - (m - log2 B) */
static orc_ct* cheb_node(orc_ctx* c, orc_ct** T, int B, int lb, const double* cf, int m, double target) {
  int n = 1 << m;
  if (n <= B) {
    double pre = target * (double)c->mod[lb];
    orc_ct* acc = cheb_combination(c, T, cf, n, lb, pre);
    rescale_inplace(c, acc);
    acc->scale = target;
    op_add_const_inplace(c, acc, cf[0]);
    return acc;
  }
  int h = n / 2;
  double* q = (double*)xcalloc(h, sizeof(double));
  double* r = (double*)xcalloc(h, sizeof(double));
  q[0] = cf[h];
  r[0] = cf[0];
  for (int j = 1; j < h; ++j) {
    q[j] = 2.0 * cf[h + j];
    r[j] = cf[j] - cf[2 * h - j];
  }
  int mb = 0;
  while ((1 << mb) < B) ++mb;
  int lq = lb - 1 - (m - 1 - mb);           /* level of the children */
  double tq = target * (double)c->mod[lq];
  tq = tq / T[h]->scale;
  orc_ct* qc = cheb_node(c, T, B, lb, q, m - 1, tq);
  orc_ct* g = ct_copy(c, T[h], lq);
  orc_ct3* t3 = op_tensor(c, qc, g);
  orc_ct* A;
  if (h <= B) {
    A = cheb_combination(c, T, r, h, lq, t3->scale);
  } else {
    orc_ct* rc = cheb_node(c, T, B, lb, r, m - 1, ldexp(1.0, c->log_scale));
    A = op_lincomb(c, rc, 1.0, NULL, 0.0, t3->scale, 0);
    ct_free(rc);
  }
  op_add3_ct_inplace(c, t3, A);
  orc_ct* out = op_relin3(c, t3);
  rescale_inplace(c, out);
  out->scale = target;
  if (h <= B) op_add_const_inplace(c, out, r[0]);
  ct_free(qc); ct_free(g); ct_free(A); ct3_free(t3);
  free(q); free(r);
  return out;
}

/* T_j by the product rules above */
static void cheb_basis_step(orc_ctx* c, orc_ct** T, orc_ct** T2, int j) {
  int a = 1;
  while (2 * a < j) a *= 2;
  int b = j - a;
  if (b == a) {
    orc_ct* P = op_square_exact(c, T[a]);
    T[j] = op_double(c, P);
    ct_free(P);
    op_add_const_inplace(c, T[j], -1.0);
  } else {
    if (!T2[a]) T2[a] = op_double(c, T[a]);
    orc_ct3* t3 = op_tensor(c, T2[a], T[b]);
    orc_ct* lo = ct_copy(c, T[a - b], t3->level);
    orc_ct* A = op_lincomb(c, lo, -1.0, NULL, 0.0, t3->scale, 0);
    op_add3_ct_inplace(c, t3, A);
    T[j] = op_relin3(c, t3);
    rescale_inplace(c, T[j]);
    ct3_free(t3); ct_free(lo); ct_free(A);
  }
}

static orc_ct* eval_mod(orc_ctx* c, const orc_ct* u) {
  double delta = ldexp(1.0, c->log_scale);
  int deg = c->boot_deg;
  int k = 0;
  while ((1 << k) < deg + 1) ++k;
  int mb = (k + 1) / 2;
  if (mb < 1) mb = 1;
  int B = 1 << mb;
  orc_ct** T = (orc_ct**)xcalloc(deg + 2, sizeof(orc_ct*));
  orc_ct** T2 = (orc_ct**)xcalloc(deg + 2, sizeof(orc_ct*));
  T[1] = ct_copy(c, u, u->level);
  for (int j = 2; j < B; ++j) cheb_basis_step(c, T, T2, j);
  for (int h = B; h < (1 << k); h *= 2) cheb_basis_step(c, T, T2, h);
  int lb = B > 2 ? T[B - 1]->level : T[1]->level;
  orc_ct* acc = cheb_node(c, T, B, lb, c->boot_cheb, k, delta);
  for (int j = 0; j <= deg + 1; ++j) { ct_free(T[j]); ct_free(T2[j]); }
  free(T); free(T2);
  for (int i = 0; i < c->boot_r; ++i) {
    orc_ct* P = op_square_exact(c, acc);
    orc_ct* y = op_double(c, P);
    ct_free(P);
    op_add_const_inplace(c, y, -1.0);
    ct_free(acc);
    acc = y;
  }
  return acc;
}
ORC_API void* orc_eval_mod(void* h, const void* u) { return eval_mod((orc_ctx*)h, (const orc_ct*)u); }

static int boot_levels(orc_ctx* c) {
  int k = 0;
  while ((1 << k) < c->boot_deg + 1) ++k;
  return 2 * c->boot_groups + k + 1 + c->boot_r;
}

/* the linear transforms: all groups of one direction, each at the level below
   the previous (targets Delta) */
/* output scale of group g: CoeffToSlot keeps 2^5 Delta until its last group
   (its first groups carry the large ModRaise overflow, so their plaintexts
   get the larger scale), everything else Delta */
static double boot_group_target(orc_ctx* c, int inverse, int g, int groups) {
  if (inverse && g < groups - 1) return ldexp(1.0, c->log_scale + 5);
  return ldexp(1.0, c->log_scale);
}
static orc_ct* boot_transform_ns(orc_ctx* c, const orc_ct* x, int inverse, int ns, int groups) {
  orc_ct* y = ct_copy(c, x, x->level);
  int l0 = x->level;
  for (int g = 0; g < groups; ++g) {
    boot_group G = boot_make_group_ns(c, inverse, g, l0 - g, ns, groups);
    orc_ct* t = boot_apply_group(c, &G, g, y, boot_group_target(c, inverse, g, groups));
    dm_free(&G.M);
    ct_free(y);
    y = t;
  }
  return y;
}
static orc_ct* boot_transform(orc_ctx* c, const orc_ct* x, int inverse) {
  return boot_transform_ns(c, x, inverse, c->n / 2, c->boot_groups);
}
static orc_ct* coeff_to_slot(orc_ctx* c, const orc_ct* x) { return boot_transform(c, x, 1); }
static orc_ct* slot_to_coeff(orc_ctx* c, const orc_ct* x) { return boot_transform(c, x, 0); }
ORC_API void* orc_boot_transform(void* h, const void* x, int inverse) {
  return boot_transform((orc_ctx*)h, (const orc_ct*)x, inverse);
}

/* the full pipeline after the scale-down: a level-0 ciphertext at scale
   q_0 / 2^ratio through ModRaise, CoeffToSlot, the split into real and
   imaginary parts, EvalMod on each, their join and SlotToCoeff */
static orc_ct* boot_core_full(orc_ctx* c, const orc_ct* x0) {
  orc_ct* y0 = mod_raise(c, x0);
  orc_ct* y = coeff_to_slot(c, y0);
  ct_free(y0);
  /* real and imaginary parts: w + conj(w), -i (w - conj(w)) */
  orc_ct* yc = op_rotate(c, y, CONJ_STEP);
  orc_ct* re = op_add(c, y, yc, 0);
  orc_ct* df = op_add(c, y, yc, 1);
  orc_ct* im = op_mul_monomial_half(c, df, 1);
  ct_free(yc); ct_free(df); ct_free(y);
  orc_ct* re2 = eval_mod(c, re);
  orc_ct* im2 = eval_mod(c, im);
  ct_free(re); ct_free(im);
  orc_ct* imi = op_mul_monomial_half(c, im2, 0);
  orc_ct* w = op_add(c, re2, imi, 0);
  ct_free(re2); ct_free(im2); ct_free(imi);
  orc_ct* w2 = slot_to_coeff(c, w);
  ct_free(w);
  if (w2->level != c->boot_out_level) die("bootstrap: level plan mismatch");
  return w2;
}

/* the whole bootstrap of a ciphertext at level >= 1 with slot values |z| <= 1;
   the result is at boot_out_level with scale Delta */
static orc_ct* bootstrap(orc_ctx* c, const orc_ct* x) {
  if (c->boot_out_level < 0) die("bootstrap: not set up");
  if (x->level < 1) die("bootstrap: input needs level >= 1");
  double tb = ldexp((double)c->mod[0], -c->boot_ratio);
  orc_ct* x1 = ct_copy(c, x, 1);
  orc_ct* x0 = op_lincomb(c, x1, 1.0, NULL, 0.0, tb, 1);
  ct_free(x1);
  orc_ct* w = boot_core_full(c, x0);
  ct_free(x0);
  c->counters[CNT_REFRESH]++;
  return w;
}
ORC_API void* orc_bootstrap(void* h, const void* x) { return bootstrap((orc_ctx*)h, (const orc_ct*)x); }

/* x + RotL(x, n) + RotL(x, 2n) + ... over every multiple of n: the trace onto
   the subring Z[X^(N/2n)], whose slot vectors repeat with period n */
static orc_ct* boot_subsum(orc_ctx* c, orc_ct* x, int n) {
  for (int64_t r = n; r < c->n / 2; r *= 2) {
    orc_ct* y = op_rotate(c, x, r);
    orc_ct* z = op_add(c, x, y, 0);
    ct_free(x);
    ct_free(y);
    x = z;
  }
  return x;
}

/* Group g of the sparse-slot transforms (n = boot_sparse slots, 'groups'
   groups like the full ones), on n-periodic slot vectors, except:
     the last CoeffToSlot group writes [w, 0] with period 2n: its diagonals
       are those of the n-slot map on the lower n slots of each 2n period
       and zero on the upper ones;
     the first SlotToCoeff group reads u = [a, b] with period 2n and applies
       the n-slot map to a + i b: each n-slot diagonal d becomes the 2n-slot
       diagonals d and d + n, whose entry at p is D[d][p mod n] times 1 or i
       as the slot it reads lies in the lower or the upper half. */
static boot_group boot_make_group_sparse(orc_ctx* c, int inverse, int g, int level) {
  int n = c->boot_sparse, groups = c->boot_groups;
  boot_group G = boot_make_group_ns(c, inverse, g, level, n, groups);
  int mask = inverse && g == groups - 1, join = !inverse && g == 0;
  if (!mask && !join) return G;
  int n2 = 2 * n;
  diagmat M2 = dm_new(n2);
  for (int d = 0; d < n; ++d) {
    if (!G.M.d[d]) continue;
    for (int p = 0; p < n2; ++p) {
      cq v = G.M.d[d][p % n];
      if (mask) {
        /* offset d or d - n read the same slot of an n-periodic input: keep
           the centred one, so the offsets stay those of the n-slot map */
        int off = d < n / 2 ? d : d + n;
        if (p < n) dm_at(&M2, off)[p] = v;
        else dm_at(&M2, off);
      } else {
        for (int k = 0; k < 2; ++k) {
          int off = (d + k * n) % n2;
          int r = (p + off) % n2;
          cq w = r < n ? v : (cq){-v.im, v.re};   /* times i on the upper half */
          cq* dst = dm_at(&M2, off);
          dst[p].re += w.re;
          dst[p].im += w.im;
        }
      }
    }
  }
  dm_free(&G.M);
  G.M = M2;
  G.ns = n2;
  G.E = n2 / G.delta;
  return G;
}

/* the sparse-slot CoeffToSlot (inverse = 1) or SlotToCoeff: every group, one level each */
static orc_ct* boot_transform_sparse(orc_ctx* c, const orc_ct* x, int inverse) {
  orc_ct* y = ct_copy(c, x, x->level);
  int l0 = x->level;
  for (int g = 0; g < c->boot_groups; ++g) {
    boot_group G = boot_make_group_sparse(c, inverse, g, l0 - g);
    orc_ct* t = boot_apply_group(c, &G, g, y, boot_group_target(c, inverse, g, c->boot_groups));
    dm_free(&G.M);
    ct_free(y);
    y = t;
  }
  return y;
}

/* Sparse-slot bootstrap (n = boot_sparse slots, 2n <= N/2; the trace and the
   n-slot transforms of Cheon, Han, Kim, Kim, Song 2018): only slots [0, n) of
   the input count, and the output repeats them with period n.
     scale-down   the constant of the full pipeline becomes the mask of
                  slots [0, n), at the same level;
     trace        at level 0, the sum over rotations by multiples of n makes
                  the message a polynomial in Y = X^(N/2n) (slots of period
                  n), so that it is unchanged by the trace after ModRaise;
     ModRaise     t = m + q_0 I; the trace again (log2(N/2n) rotations)
                  leaves (N/2n) (m + q_0 I'), I' the part of I in Z[Y];
     CoeffToSlot  the n-slot special FFT (root zeta^(N/2n) of order 4n) with
                  n/(N/2) folded into its first group; the last group writes
                  [w, 0] with period 2n;
     split        [re, 0] = w + conj(w), [im, 0] = -i (w - conj(w)), and
                  u = [re, 0] + RotR([im, 0], n) = [re, im]: real parts in
                  slots [0, n), imaginary parts in [n, 2n) of each period;
     EvalMod      as in the full pipeline, once for both parts;
     SlotToCoeff  the n-slot transform of re + i im, the first group
                  reading the two halves.
   Same depth as the full pipeline, so the same output level. */
static orc_ct* bootstrap_sparse(orc_ctx* c, const orc_ct* x) {
  int ns = c->boot_sparse, S = c->n / 2;
  if (c->boot_out_level < 0 || ns <= 0) die("bootstrap_sparse: not set up");
  if (x->level < 1) die("bootstrap: input needs level >= 1");
  double tb = ldexp((double)c->mod[0], -c->boot_ratio);
  double* mask = (double*)xcalloc(ns, sizeof(double));
  for (int j = 0; j < ns; ++j) mask[j] = 1.0;
  orc_ct* x1 = ct_copy(c, x, 1);
  orc_ct* x0 = op_mul_plain(c, x1, mask, ns, tb);
  ct_free(x1);
  free(mask);
  x0 = boot_subsum(c, x0, ns);
  orc_ct* y0 = mod_raise(c, x0);
  ct_free(x0);
  y0 = boot_subsum(c, y0, ns);
  orc_ct* w = boot_transform_sparse(c, y0, 1);
  ct_free(y0);
  orc_ct* wc = op_rotate(c, w, CONJ_STEP);
  orc_ct* re = op_add(c, w, wc, 0);
  orc_ct* df = op_add(c, w, wc, 1);
  orc_ct* im = op_mul_monomial_half(c, df, 1);
  ct_free(w); ct_free(wc); ct_free(df);
  orc_ct* imr = op_rotate(c, im, (int64_t)S - ns);
  orc_ct* u = op_add(c, re, imr, 0);
  ct_free(re); ct_free(im); ct_free(imr);
  orc_ct* e = eval_mod(c, u);
  ct_free(u);
  orc_ct* out = boot_transform_sparse(c, e, 0);
  ct_free(e);
  if (out->level != c->boot_out_level) die("bootstrap_sparse: level plan mismatch");
  c->counters[CNT_REFRESH]++;
  return out;
}
ORC_API void* orc_bootstrap_sparse(void* h, const void* x) {
  return bootstrap_sparse((orc_ctx*)h, (const orc_ct*)x);
}
/* Window-packed bootstrap: a refresh of k single-query ciphertexts that each
   read only slots [0, W) afterwards (W = boot_sparse) shares full-slot
   bootstraps.  A design of this implementation (the method bootstraps each
   ciphertext); groups of m <= N/2W inputs in order, each group:
     scale-down   as in the sparse-slot bootstrap: the mask of slots [0, W)
                  at scale q_0 / 2^ratio, down to level 0, giving v_j;
     pack         T = sum_i RotL(z_i, i W) with z_i = v_(m-1-i), by pairs:
                  at round b, node t = node 2t + RotL(node 2t+1, 2^b W)
                  (an odd last node passes through); then
                  P = RotL(T, ((N/2W - m + 1) mod N/2W) W), one rotation by
                  2^b W for each set bit b, lowest first.  P holds v_j's
                  slots [0, W) at [jW, jW + W) and zeros elsewhere;
     bootstrap    the full pipeline from ModRaise on (boot_core_full);
     unpack       U_0 = P'; at round b = 0, 1, ... every U_o with o < 2^b
                  gives U_(o + 2^b) = RotL(U_o, 2^b W) while o + 2^b < m, so
                  U_j = RotL(P', j W) holds input j's slots [0, W) at [0, W)
                  (and the other inputs' windows elsewhere).
   Every rotation is by a power-of-two multiple of W below N/2, the same
   steps as the sparse-slot trace, so no other key is needed. */
static void bootstrap_packed(orc_ctx* c, orc_ct* const* xs, int k, orc_ct** out) {
  int W = c->boot_sparse, S = c->n / 2;
  if (c->boot_out_level < 0 || W <= 0) die("bootstrap_packed: not set up");
  int per = S / W;
  double tb = ldexp((double)c->mod[0], -c->boot_ratio);
  double* mask = (double*)xcalloc(W, sizeof(double));
  for (int j = 0; j < W; ++j) mask[j] = 1.0;
  for (int p0 = 0; p0 < k; p0 += per) {
    int m = k - p0 < per ? k - p0 : per;
    orc_ct** z = (orc_ct**)xcalloc(m, sizeof(orc_ct*));
    for (int i = 0; i < m; ++i) {
      const orc_ct* x = xs[p0 + m - 1 - i];
      if (x->level < 1) die("bootstrap: input needs level >= 1");
      orc_ct* x1 = ct_copy(c, x, 1);
      z[i] = op_mul_plain(c, x1, mask, W, tb);
      ct_free(x1);
    }
    int cnt = m;
    for (int b = 0; cnt > 1; ++b) {
      int nc = 0;
      for (int t = 0; 2 * t < cnt; ++t) {
        if (2 * t + 1 < cnt) {
          orc_ct* r = op_rotate(c, z[2 * t + 1], (int64_t)W << b);
          orc_ct* u = op_add(c, z[2 * t], r, 0);
          ct_free(r);
          ct_free(z[2 * t]);
          ct_free(z[2 * t + 1]);
          z[nc++] = u;
        } else {
          z[nc++] = z[2 * t];
        }
      }
      cnt = nc;
    }
    orc_ct* P = z[0];
    int shift = (per - m + 1) % per;
    for (int b = 0; (1 << b) <= shift; ++b)
      if (shift & (1 << b)) {
        orc_ct* r = op_rotate(c, P, (int64_t)W << b);
        ct_free(P);
        P = r;
      }
    orc_ct* Pb = boot_core_full(c, P);
    ct_free(P);
    orc_ct** u = out + p0;
    u[0] = Pb;
    for (int b = 0; (1 << b) < m; ++b)
      for (int o = 0; o < (1 << b) && o + (1 << b) < m; ++o) u[o + (1 << b)] = op_rotate(c, u[o], (int64_t)W << b);
    free(z);
    c->counters[CNT_REFRESH] += m;
  }
  free(mask);
}
ORC_API void orc_bootstrap_packed(void* h, void* const* xs, int k, void** out) {
  bootstrap_packed((orc_ctx*)h, (orc_ct* const*)xs, k, (orc_ct**)out);
}

/* the sparse-slot bootstrap keeps slots [0, n): n a power of two with
   2n <= N/2 and at least one radix-2 stage per group; 0 turns it off.
   Returns 0, or -1 for an n it cannot take. */
ORC_API int orc_set_boot_sparse(void* h, int n) {
  orc_ctx* c = (orc_ctx*)h;
  c->boot_sparse = 0;
  if (n == 0) return 0;
  int L = 0;
  while ((1 << L) < n) ++L;
  if (c->boot_out_level < 0 || n < 0 || (n & (n - 1)) || 2 * n > c->n / 2 || L < c->boot_groups) return -1;
  c->boot_sparse = n;
  return 0;
}

/* bootstrapping parameters; call before keygen (the secret weight h is used
   there).  mode 1 makes every refresh a bootstrap.  Returns the level of a
   bootstrapped ciphertext, or -1 when the chain is too short. */
ORC_API int orc_set_boot(void* h, int secret_h, int K, int r, int deg, int ratio, int groups, int mode) {
  orc_ctx* c = (orc_ctx*)h;
  c->secret_h = secret_h;
  c->boot_sparse = 0;
  if (c->boot_mode) c->refresh_level = c->refresh_level_set;
  if (K <= 0) { c->boot_out_level = -1; c->boot_mode = 0; return -1; }
  if (deg < 1 || ((deg + 1) & deg) || r < 0 || groups < 1 || ratio < 1) die("bad bootstrapping parameters");
  c->boot_K = K; c->boot_r = r; c->boot_deg = deg; c->boot_ratio = ratio; c->boot_groups = groups;
  free(c->boot_cheb);
  c->boot_cheb = (double*)xcalloc(deg + 1, sizeof(double));
  boot_cheb_coeffs(K, r, deg, c->boot_cheb);
  int out = c->n_q - 1 - boot_levels(c);
  if (out < c->min_level) { c->boot_out_level = -1; c->boot_mode = 0; c->refresh_level = c->refresh_level_set; return -1; }
  c->boot_out_level = out;
  c->boot_mode = mode;
  if (mode) c->refresh_level = out;
  return out;
}

/* the CoeffToSlot (inverse = 1) or SlotToCoeff group g as its slot map applied
   to v (complex, S values), for checks against the matrix definition */
ORC_API void orc_boot_group_apply(void* h, int inverse, int g, const double* vre, const double* vim, double* ore,
                                  double* oim) {
  orc_ctx* c = (orc_ctx*)h;
  int S = c->n / 2;
  boot_group G = boot_make_group(c, inverse, g, 0);
  for (int p = 0; p < S; ++p) {
    __float128 ar = 0, ai = 0;
    for (int d = 0; d < S; ++d) {
      if (!G.M.d[d]) continue;
      cq v = {vre[(p + d) % S], vim[(p + d) % S]};
      cq t = cq_mul(G.M.d[d][p], v);
      ar += t.re;
      ai += t.im;
    }
    ore[p] = (double)ar;
    oim[p] = (double)ai;
  }
  dm_free(&G.M);
}
/* the sparse-slot CoeffToSlot (inverse = 1) or SlotToCoeff, every group, as
   slot maps applied to v (2n complex values: one 2n period of the slots) */
ORC_API void orc_boot_sparse_apply(void* h, int inverse, const double* vre, const double* vim, double* ore,
                                   double* oim) {
  orc_ctx* c = (orc_ctx*)h;
  int n2 = 2 * c->boot_sparse;
  cq* v = (cq*)xcalloc(n2, sizeof(cq));
  cq* o = (cq*)xcalloc(n2, sizeof(cq));
  for (int p = 0; p < n2; ++p) v[p] = (cq){vre[p], vim[p]};
  for (int g = 0; g < c->boot_groups; ++g) {
    boot_group G = boot_make_group_sparse(c, inverse, g, 0);
    for (int p = 0; p < n2; ++p) {
      __float128 ar = 0, ai = 0;
      for (int d = 0; d < G.ns; ++d) {
        if (!G.M.d[d]) continue;
        cq t = cq_mul(G.M.d[d][p % G.ns], v[(p + d) % n2]);
        ar += t.re;
        ai += t.im;
      }
      o[p] = (cq){ar, ai};
    }
    memcpy(v, o, sizeof(cq) * (size_t)n2);
    dm_free(&G.M);
  }
  for (int p = 0; p < n2; ++p) { ore[p] = (double)v[p].re; oim[p] = (double)v[p].im; }
  free(v);
  free(o);
}
ORC_API void* orc_boot_transform_sparse(void* h, const void* x, int inverse) {
  return boot_transform_sparse((orc_ctx*)h, (const orc_ct*)x, inverse);
}
ORC_API void* orc_mod_raise(void* h, const void* x) { return mod_raise((orc_ctx*)h, (const orc_ct*)x); }
ORC_API void* orc_mul_monomial_half(void* h, const void* x, int neg) {
  return op_mul_monomial_half((orc_ctx*)h, (const orc_ct*)x, neg);
}
ORC_API int orc_boot_out_level(void* h) { return ((orc_ctx*)h)->boot_out_level; }
