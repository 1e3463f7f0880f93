// The encrypted Argmax of arXiv 2502.00847 (Sec. 3.2, Algorithm 1) as a
// batched program: each query is a sequence of steps; every round runs one
// step kind for all queries waiting on it, in the same kernel launches.
#include <math.h>

#include <algorithm>

#include "runtime.h"

namespace secpe {

// Sign polynomials (Eq. 4), odd coefficients of x, x^3, x^5, x^7, x^9.
// f is the closed form sum_{i<=4} C(2i,i) 4^-i x (1-x^2)^i; g is the degree-9
// g of Cheon, Kim and Kim (ASIACRYPT 2020).  The paper fixes only "degree 9".
static const double kSignF[5] = {315.0 / 128.0, -420.0 / 128.0, 378.0 / 128.0, -180.0 / 128.0, 35.0 / 128.0};
static const double kSignG[5] = {5850.0 / 1024.0, -34974.0 / 1024.0, 97015.0 / 1024.0, -113492.0 / 1024.0,
                                 46623.0 / 1024.0};

enum StepKind { S_ROTADD = 0, S_NORMALISE, S_DUP, S_MAXPRE, S_POLY, S_MAXPOST, S_FINALPRE, S_FINALPOST, S_NKINDS };

struct Step {
  int kind;
  int arg;     // ROTADD: rotation; MAXPRE: QuickMax index i; POLY: polynomial index in the Sign
  bool max;    // POLY: part of a Max step (true) or the final Sign (false)
};

struct QState {
  ArgmaxQuery* q;
  int kp, cp, lk, lc;
  int bsz = 0;   // packed input: block size (0 = one query per ciphertext)
  uint64_t rnext = 0;
  CT y, ydup, ym, d, s, x;
  int lp = 0, ls = 0;
  double t_sign = 0.0;
  std::vector<Step> prog;
  size_t pc = 0;
};

static void free_owned(Builder& b, CT& x) {
  if (x.slot >= 0) b.free_ct(x);
  x = CT{};
}

static CT view(const CT& x) {
  CT v = x;
  v.slot = -1;
  return v;
}

// refresh, in one batch, every item whose level cannot afford 'need' more levels
static void maybe_refresh(Builder& b, std::vector<QState*>& qs, std::vector<CT*> cts, const std::vector<int>& need) {
  std::vector<CT> in;
  std::vector<uint64_t> seed, index;
  std::vector<size_t> who;
  std::vector<int> span;
  const int top = b.C.refresh_level;
  for (size_t i = 0; i < qs.size(); ++i) {
    CT& x = *cts[i];
    if (x.level - need[i] >= b.C.min_level) continue;
    if (top - need[i] < b.C.min_level) { b.fail(-3, "modulus chain too short for one unit"); return; }
    in.push_back(x);
    seed.push_back(qs[i]->q->refresh_seed);
    index.push_back(qs[i]->rnext++);
    who.push_back(i);
    // after Eq. 5 a single query reads only slots [0, 2C') again (the
    // duplicate of line 2 and every QuickMax window stay inside)
    span.push_back(qs[i]->bsz ? 0 : 2 * qs[i]->cp);
  }
  if (in.empty()) return;
  std::vector<CT> out = b.refresh(in, seed, index, &span);
  if (b.err_code) return;
  for (size_t k = 0; k < who.size(); ++k) {
    CT& x = *cts[who[k]];
    free_owned(b, x);
    x = out[k];
  }
}

static void run_step(Builder& b, int kind, std::vector<QState*>& qs) {
  Ctx& C = b.C;
  const double delta = ldexp(1.0, C.log_scale);
  const int slots = C.N / 2;
  const int total = C.dg + C.df;
  const size_t n = qs.size();
  std::vector<std::pair<CT, CT>> pr;
  switch (kind) {
    case S_ROTADD: {  // prompt sum by doubling: y <- y + RotL(y, C' 2^i)
      std::vector<CT> in;
      std::vector<int64_t> st;
      for (QState* s : qs) { in.push_back(s->y); st.push_back(s->prog[s->pc].arg); }
      std::vector<CT> r = b.rotate(in, st);
      if (b.err_code) return;
      for (size_t i = 0; i < n; ++i) pr.push_back({qs[i]->y, r[i]});
      std::vector<CT> y = b.add(pr, false);
      if (b.err_code) return;
      for (size_t i = 0; i < n; ++i) {
        b.free_ct(r[i]);
        free_owned(b, qs[i]->y);
        qs[i]->y = y[i];
      }
      break;
    }
    case S_NORMALISE: {  // Eq. 5 on [0, C): mask * (y - D_min) / (D_max - D_min)
      std::vector<CT*> cts;
      for (QState* s : qs) cts.push_back(&s->y);
      maybe_refresh(b, qs, cts, std::vector<int>(n, 1));
      if (b.err_code) return;
      std::vector<QState*> one, packed;
      for (QState* s : qs) (s->bsz ? packed : one).push_back(s);
      if (!one.empty()) {
        std::vector<CT> in;
        std::vector<double> v;
        for (QState* s : one) { in.push_back(s->y); v.push_back(-s->q->d_min); }
        std::vector<CT> y1 = b.add_const(in, v);
        if (b.err_code) return;
        std::vector<std::vector<double>> masks;
        std::vector<double> tg;
        for (QState* s : one) {
          std::vector<double> m(s->cp, 0.0);
          const double inv_range = 1.0 / (s->q->d_max - s->q->d_min);
          for (int j = 0; j < s->q->C; ++j) m[j] = inv_range;
          masks.push_back(m);
          tg.push_back(delta);
        }
        std::vector<CT> yn = b.mul_plain(y1, masks, tg);
        if (b.err_code) return;
        for (size_t i = 0; i < one.size(); ++i) {
          b.free_ct(y1[i]);
          free_owned(b, one[i]->y);
          one[i]->y = yn[i];
        }
      }
      if (!packed.empty()) {
        // per block b: -D_min_b on its classes, then the mask 1/(D_max_b - D_min_b) there
        std::vector<CT> in;
        std::vector<Builder::SparseSlots> shift, mask;
        std::vector<double> tg;
        for (QState* s : packed) {
          Builder::SparseSlots sh, mk;
          const ArgmaxQuery& q = *s->q;
          for (size_t bl = 0; bl < q.bK.size(); ++bl) {
            const double inv_range = 1.0 / (q.bhi[bl] - q.blo[bl]);
            for (int j = 0; j < q.bC[bl]; ++j) {
              const int slot = (int)bl * s->bsz + j;
              sh.slot.push_back(slot);
              sh.val.push_back(-q.blo[bl]);
              mk.slot.push_back(slot);
              mk.val.push_back(inv_range);
            }
          }
          in.push_back(s->y);
          shift.push_back(sh);
          mask.push_back(mk);
          tg.push_back(delta);
        }
        std::vector<CT> y1 = b.add_plain_sparse(in, shift);
        if (b.err_code) return;
        std::vector<CT> yn = b.mul_plain_sparse(y1, mask, tg);
        if (b.err_code) return;
        for (size_t i = 0; i < packed.size(); ++i) {
          b.free_ct(y1[i]);
          free_owned(b, packed[i]->y);
          packed[i]->y = yn[i];
        }
      }
      break;
    }
    case S_DUP: {  // Algorithm 1, line 2: y <- y + RotR(y, n), n = C'
      std::vector<CT> in;
      std::vector<int64_t> st;
      for (QState* s : qs) { in.push_back(s->y); st.push_back((int64_t)slots - s->cp); }
      std::vector<CT> r = b.rotate(in, st);
      if (b.err_code) return;
      for (size_t i = 0; i < n; ++i) pr.push_back({qs[i]->y, r[i]});
      std::vector<CT> y = b.add(pr, false);
      if (b.err_code) return;
      for (size_t i = 0; i < n; ++i) {
        b.free_ct(r[i]);
        free_owned(b, qs[i]->y);
        qs[i]->ydup = y[i];
        qs[i]->ym = view(y[i]);
      }
      break;
    }
    case S_MAXPRE: {  // QuickMax step i: r = RotL(y, 2^i); d = r - y; s = r + y  (Eq. 6)
      std::vector<CT*> cts;
      for (QState* s : qs) cts.push_back(&s->ym);
      maybe_refresh(b, qs, cts, std::vector<int>(n, 1));
      if (b.err_code) return;
      std::vector<CT> in;
      std::vector<int64_t> st;
      for (QState* s : qs) { in.push_back(s->ym); st.push_back((int64_t)1 << s->prog[s->pc].arg); }
      std::vector<CT> r = b.rotate(in, st);
      if (b.err_code) return;
      for (size_t i = 0; i < n; ++i) pr.push_back({r[i], qs[i]->ym});
      std::vector<CT> d, sm;
      b.add_sub(pr, d, sm);
      if (b.err_code) return;
      for (size_t i = 0; i < n; ++i) {
        QState* s = qs[i];
        b.free_ct(r[i]);
        free_owned(b, s->ym);
        s->d = d[i];
        s->s = sm[i];
        s->x = view(d[i]);
        // level plan of the Sign so that d * Sign/2 lands on the scale delta
        int lvl = s->d.level;
        for (int j = 0; j < total; ++j) {
          const int need = 4 + (j == total - 1 ? 1 : 0);
          if (lvl - need < C.min_level) lvl = C.refresh_level;
          if (lvl - need < C.min_level) { b.fail(-3, "modulus chain too short for one unit"); return; }
          lvl -= 4;
        }
        s->ls = lvl;
        s->lp = std::min(s->d.level, lvl);
        double t = delta * (double)C.mod[s->lp];
        t = t / s->d.scale;
        s->t_sign = t;
      }
      b.counters[6] += (int64_t)n;
      break;
    }
    case S_POLY: {  // one polynomial of Sign = f^df(g^dg(x))  (Eq. 4)
      std::vector<CT*> cts;
      std::vector<int> need;
      for (QState* s : qs) {
        const Step& st = s->prog[s->pc];
        cts.push_back(&s->x);
        need.push_back(4 + ((st.max && st.arg == total - 1) ? 1 : 0));
      }
      maybe_refresh(b, qs, cts, need);
      if (b.err_code) return;
      std::vector<CT> in;
      std::vector<const double*> coef;
      std::vector<double> gain, tg;
      for (QState* s : qs) {
        const Step& st = s->prog[s->pc];
        const bool last = st.arg == total - 1;
        if (last && st.max && s->x.level - 4 != s->ls) { b.fail(-1, "level plan mismatch"); return; }
        in.push_back(s->x);
        coef.push_back(st.arg < C.dg ? kSignG : kSignF);
        gain.push_back(last && st.max ? 0.5 : 1.0);
        tg.push_back(last && st.max ? s->t_sign : delta);
      }
      std::vector<CT> y = b.eval_odd9(in, coef, gain, tg);
      if (b.err_code) return;
      for (size_t i = 0; i < n; ++i) {
        free_owned(b, qs[i]->x);
        qs[i]->x = y[i];
        if (qs[i]->prog[qs[i]->pc].arg == total - 1) b.counters[0]++;
      }
      break;
    }
    case S_MAXPOST: {  // Max = (a+b)/2 + (a-b)/2 * Sign(a-b)   (Eq. 6)
      // d * Sign/2 as a degree-2 ciphertext with (a+b)/2 added at the same
      // scale, then one relinearise-and-rescale
      auto lower = [](CT x, int l) { x.level = l; x.slot = -1; return x; };
      std::vector<Builder::LinItem> li;
      for (QState* s : qs) {
        Builder::LinItem t{};
        t.a = lower(s->s, s->lp);
        t.va = 0.5;
        t.target = s->d.scale * s->x.scale;
        li.push_back(t);
      }
      const size_t mark = b.scratch_mark();
      std::vector<Builder::TensorItem> ti;
      for (size_t i = 0; i < n; ++i) {
        Builder::TensorItem t{};
        t.a = lower(qs[i]->d, qs[i]->lp);
        t.b = lower(qs[i]->x, qs[i]->lp);
        t.fl = li[i];   // (a+b)/2 formed inside the degree-2 sum
        t.has_fl = true;
        ti.push_back(t);
      }
      std::vector<Builder::Deg2> d2 = b.tensor2(ti);
      if (b.err_code) return;
      std::vector<CT> out = b.relin_rescale(d2);
      if (b.err_code) return;
      b.scratch_release(mark);
      for (size_t i = 0; i < n; ++i) {
        QState* s = qs[i];
        free_owned(b, s->d);
        free_owned(b, s->s);
        free_owned(b, s->x);
        s->ym = out[i];
      }
      break;
    }
    case S_FINALPRE: {  // Algorithm 1, line 4: y <- y - y_max
      for (QState* s : qs) pr.push_back({s->ydup, s->ym});
      std::vector<CT> d = b.add(pr, true);
      if (b.err_code) return;
      for (size_t i = 0; i < n; ++i) {
        QState* s = qs[i];
        free_owned(b, s->ym);
        free_owned(b, s->ydup);
        s->d = d[i];
        s->x = view(d[i]);
      }
      break;
    }
    case S_FINALPOST: {  // lines 5-6: z <- Sign(y) + 1, written to the caller's buffer
      std::vector<EwJob> j;
      for (QState* s : qs) {
        const CT& x = s->x;
        double kf = 1.0 * x.scale;
        const int64_t K = llround(kf);
        EwJob e{};
        e.o0 = s->q->out.d;
        e.o1 = s->q->out.d + (size_t)C.n_q * C.N;
        e.a0 = b.c0(x);
        e.a1 = b.c1(x);
        e.k = b.put_residues(K, x.level + 1);
        e.n_limbs = x.level + 1;
        e.n_chain = x.level + 1;
        e.op = EW_ADD_CONST;
        j.push_back(e);
        s->q->out.level = x.level;
        s->q->out.scale = x.scale;
      }
      b.ew(j);
      for (QState* s : qs) {
        free_owned(b, s->x);
        free_owned(b, s->d);
      }
      break;
    }
    default:
      break;
  }
}

// ---------------------------------------------------------------------------
// The comparison path the paper measures against (Phoenix, Sec. 3.2): after
// the prompt sum and Eq. 5, s = sum_{i<C} Sign(y - RotL(y, i)) with y
// duplicated at offset C, then z = (Sign((s - (C-2)) / (2C-3)) + 1) / 2.  The
// C-1 comparisons are independent and run in the same launches.  The k-th
// refresh of comparison i (i = 0: the prefix and the final Sign) uses refresh
// index k * 512 + i.
// ---------------------------------------------------------------------------
static const int kPhoenixStride = 512;

// refresh every chain whose level cannot afford 'need'; chain i's k-th refresh
// takes index k * 512 + chain[i]
static void refresh_chains(Builder& b, std::vector<CT>& x, const std::vector<int>& chain, std::vector<int>& k,
                           int need, uint64_t seed) {
  std::vector<CT> in;
  std::vector<uint64_t> sd, idx;
  std::vector<size_t> who;
  for (size_t i = 0; i < x.size(); ++i) {
    if (x[i].level - need >= b.C.min_level) continue;
    if (b.C.refresh_level - need < b.C.min_level) { b.fail(-3, "modulus chain too short for one unit"); return; }
    in.push_back(x[i]);
    sd.push_back(seed);
    idx.push_back((uint64_t)k[i]++ * kPhoenixStride + (uint64_t)chain[i]);
    who.push_back(i);
  }
  if (in.empty()) return;
  std::vector<CT> out = b.refresh(in, sd, idx);
  if (b.err_code) return;
  for (size_t j = 0; j < who.size(); ++j) {
    free_owned(b, x[who[j]]);
    x[who[j]] = out[j];
  }
}

// Sign = f^df(g^dg(x)) on every item, each with its refresh chain
static std::vector<CT> sign_chains(Builder& b, std::vector<CT> x, const std::vector<int>& chain, std::vector<int>& k,
                                   double last_gain, uint64_t seed) {
  Ctx& C = b.C;
  const int total = C.dg + C.df;
  const double delta = ldexp(1.0, C.log_scale);
  for (int j = 0; j < total; ++j) {
    refresh_chains(b, x, chain, k, 4, seed);
    if (b.err_code) return {};
    const bool last = j == total - 1;
    std::vector<const double*> coef(x.size(), j < C.dg ? kSignG : kSignF);
    std::vector<double> gain(x.size(), last ? last_gain : 1.0), tg(x.size(), delta);
    std::vector<CT> y = b.eval_odd9(x, coef, gain, tg);
    if (b.err_code) return {};
    for (size_t i = 0; i < x.size(); ++i) free_owned(b, x[i]);
    x = y;
  }
  b.counters[0] += (int64_t)x.size();
  return x;
}

void build_phoenix(Builder& b, ArgmaxQuery& q) {
  Ctx& C = b.C;
  const double delta = ldexp(1.0, C.log_scale);
  const int slots = C.N / 2;
  const int n = q.C;
  const int lk = ilog2_ceil(q.K), cp = 1 << ilog2_ceil(n);
  if (n < 2 || n >= kPhoenixStride || (int64_t)(1 << lk) * cp > slots || 2 * n > slots) {
    b.fail(-1, "phoenix path: need 2 <= C < 512 and the shape inside the slots");
    return;
  }
  const uint64_t seed = q.refresh_seed;
  std::vector<int> chain0{0}, k0{0};
  std::vector<CT> y{view(q.in)};
  for (int i = 0; i < lk; ++i) {
    std::vector<CT> r = b.rotate(y, {(int64_t)cp << i});
    if (b.err_code) return;
    std::vector<CT> s = b.add({{y[0], r[0]}}, false);
    if (b.err_code) return;
    b.free_ct(r[0]);
    free_owned(b, y[0]);
    y = s;
  }
  refresh_chains(b, y, chain0, k0, 1, seed);
  if (b.err_code) return;
  std::vector<CT> y1 = b.add_const(y, {-q.d_min});
  if (b.err_code) return;
  std::vector<double> mask(cp, 0.0);
  for (int j = 0; j < n; ++j) mask[j] = 1.0 / (q.d_max - q.d_min);
  std::vector<CT> yn = b.mul_plain(y1, {mask}, {delta});
  if (b.err_code) return;
  b.free_ct(y1[0]);
  free_owned(b, y[0]);
  std::vector<CT> r = b.rotate(yn, {(int64_t)slots - n});
  if (b.err_code) return;
  std::vector<CT> yd = b.add({{yn[0], r[0]}}, false);
  if (b.err_code) return;
  b.free_ct(r[0]);
  b.free_ct(yn[0]);
  // the C-1 comparisons, batched
  std::vector<CT> src(n - 1, yd[0]);
  std::vector<int64_t> st;
  std::vector<int> chain, kc(n - 1, 0);
  for (int i = 1; i < n; ++i) { st.push_back(i); chain.push_back(i); }
  std::vector<CT> ri = b.rotate(src, st);
  if (b.err_code) return;
  std::vector<std::pair<CT, CT>> pr;
  for (int i = 0; i < n - 1; ++i) pr.push_back({yd[0], ri[i]});
  std::vector<CT> di = b.add(pr, true);
  if (b.err_code) return;
  for (CT& v : ri) b.free_ct(v);
  b.free_ct(yd[0]);
  std::vector<CT> si = sign_chains(b, di, chain, kc, 1.0, seed);
  if (b.err_code) return;
  CT s = si[0];
  for (int i = 1; i < n - 1; ++i) {
    std::vector<CT> t = b.add({{s, si[i]}}, false);
    if (b.err_code) return;
    free_owned(b, s);
    b.free_ct(si[i]);
    s = t[0];
  }
  std::vector<CT> sv{s};
  refresh_chains(b, sv, chain0, k0, 1, seed);
  if (b.err_code) return;
  std::vector<CT> s1 = b.add_const(sv, {-(double)(n - 2)});
  if (b.err_code) return;
  std::vector<CT> x = b.mul_const(s1, {1.0 / (double)(2 * n - 3)}, {delta});
  if (b.err_code) return;
  b.free_ct(s1[0]);
  free_owned(b, sv[0]);
  std::vector<CT> z = sign_chains(b, x, chain0, k0, 0.5, seed);
  if (b.err_code) return;
  // z + 1/2 into the caller's buffer
  const int64_t half = llround(0.5 * z[0].scale);
  EwJob e{};
  e.o0 = q.out.d;
  e.o1 = q.out.d + (size_t)C.n_q * C.N;
  e.a0 = b.c0(z[0]);
  e.a1 = b.c1(z[0]);
  e.k = b.put_residues(half, z[0].level + 1);
  e.n_limbs = z[0].level + 1;
  e.n_chain = z[0].level + 1;
  e.op = EW_ADD_CONST;
  b.ew({e});
  q.out.level = z[0].level;
  q.out.scale = z[0].scale;
  free_owned(b, z[0]);
}

void packed_shape(const std::vector<int>& K, const std::vector<int>& C, int* kp, int* cp, int* bsz) {
  int lk = 0, lc = 0;
  for (size_t i = 0; i < K.size(); ++i) {
    lk = std::max(lk, ilog2_ceil(K[i]));
    lc = std::max(lc, ilog2_ceil(C[i]));
  }
  *kp = 1 << lk;
  *cp = 1 << lc;
  *bsz = std::max(*kp * *cp, 2 * *cp);
}

ArgmaxProgram::ArgmaxProgram() {}
ArgmaxProgram::~ArgmaxProgram() {
  for (QState* s : st_) delete s;
}

size_t ArgmaxProgram::active() const { return st_.size(); }

// the step list of one query: prompt sum, normalisation, duplication, the
// QuickMax steps (each a Max of Eq. 6 around one Sign) and the final Sign + 1
bool ArgmaxProgram::add(Builder& b, ArgmaxQuery* q) {
  Ctx& C = b.C;
  const int total = C.dg + C.df;
  QState* s = new QState();
  s->q = q;
  if (!q->bK.empty()) {
    packed_shape(q->bK, q->bC, &s->kp, &s->cp, &s->bsz);
    s->lk = ilog2_ceil(s->kp);
    s->lc = ilog2_ceil(s->cp);
    if ((int64_t)q->bK.size() * s->bsz > C.N / 2) {
      delete s;
      b.fail(-1, "packed queries exceed the slot count");
      return false;
    }
  } else {
    s->lk = ilog2_ceil(q->K);
    s->lc = ilog2_ceil(q->C);
    s->kp = 1 << s->lk;
    s->cp = 1 << s->lc;
    if (q->K < 1 || q->C < 1 || (int64_t)s->kp * s->cp > C.N / 2) {
      delete s;
      b.fail(-1, "K' * C' exceeds the slot count");
      return false;
    }
  }
  s->y = view(q->in);
  for (int k = 0; k < s->lk; ++k) s->prog.push_back({S_ROTADD, s->cp << k, false});
  s->prog.push_back({S_NORMALISE, 0, false});
  s->prog.push_back({S_DUP, 0, false});
  for (int k = 0; k < s->lc; ++k) {
    s->prog.push_back({S_MAXPRE, k, true});
    for (int j = 0; j < total; ++j) s->prog.push_back({S_POLY, j, true});
    s->prog.push_back({S_MAXPOST, k, true});
  }
  s->prog.push_back({S_FINALPRE, 0, false});
  for (int j = 0; j < total; ++j) s->prog.push_back({S_POLY, j, false});
  s->prog.push_back({S_FINALPOST, 0, false});
  st_.push_back(s);
  return true;
}

std::vector<ArgmaxQuery*> ArgmaxProgram::round(Builder& b, bool all_kinds) {
  std::vector<ArgmaxQuery*> done;
  int count[S_NKINDS] = {0};
  for (QState* s : st_) count[s->prog[s->pc].kind]++;
  if (st_.empty()) return done;
  std::vector<int> kinds;
  if (all_kinds) {
    for (int k = 0; k < S_NKINDS; ++k) kinds.push_back(k);
  } else {
    int kind = 0;
    for (int k = 1; k < S_NKINDS; ++k)
      if (count[k] > count[kind]) kind = k;
    kinds.push_back(kind);
  }
  // With all_kinds the kinds run in ascending order and a query whose next
  // step is of a later kind takes it in the same round (at most one step of
  // each kind per query per round); otherwise one kind runs, one step each.
  // Either way each query's steps keep their order, so its bits do not
  // depend on the grouping.
  for (int kind : kinds) {
    std::vector<QState*> qs;
    for (QState* s : st_)
      if (s->pc < s->prog.size() && s->prog[s->pc].kind == kind) qs.push_back(s);
    if (qs.empty()) continue;
    run_step(b, kind, qs);
    if (b.err_code) return done;
    for (QState* s : qs) s->pc++;
  }
  std::vector<QState*> keep;
  for (QState* s : st_) {
    if (s->pc >= s->prog.size()) {
      done.push_back(s->q);
      delete s;
    } else {
      keep.push_back(s);
    }
  }
  st_.swap(keep);
  return done;
}

void build_argmax(Builder& b, std::vector<ArgmaxQuery>& queries) {
  ArgmaxProgram prog;
  for (ArgmaxQuery& q : queries)
    if (!prog.add(b, &q)) return;
  while (prog.active()) {
    prog.round(b, false);
    if (b.err_code) return;
  }
}

}  // namespace secpe
