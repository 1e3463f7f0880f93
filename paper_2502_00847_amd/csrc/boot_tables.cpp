// Host tables of the bootstrapping pipeline, computed in binary128 and rounded
// to binary64 (built with g++ and libquadmath):
//  * the slot vectors of the linear-transform groups: radix-2 stages of the
//    special FFT (Cheon, Han, Kim, Kim, Song, SAC 2018) on the N/2 slots
//    (slot j <-> zeta^(5^j), zeta = e^(i pi / N)), merged into groups that
//    each cost one level; CoeffToSlot applies the inverse stages m = S .. 2,
//    SlotToCoeff the forward stages m = 2 .. S; the sparse-slot transforms
//    are the same stages of the n-slot FFT (root zeta^(N/2n) of order 4n),
//    on slot vectors of period n;
//  * the Chebyshev interpolant of the scaled cosine that EvalMod evaluates
//    (Han, Ki, CT-RSA 2020).
#include <quadmath.h>

#include <map>
#include <vector>

#include "boot_tables.h"

namespace secpe {

namespace {

struct Q2 {
  __float128 re = 0, im = 0;
};
inline Q2 qmul(const Q2& a, const Q2& b) {
  Q2 r;
  r.re = a.re * b.re - a.im * b.im;
  r.im = a.re * b.im + a.im * b.re;
  return r;
}
inline bool qzero(const Q2& a) { return a.re == 0 && a.im == 0; }

// exp(i pi t / N) through cos(pi t / N) and sin(pi t / N) = cos(pi (t + 3N/2) / N)
Q2 root(uint64_t t, int n) {
  const uint64_t m2 = 2ull * (uint64_t)n;
  t %= m2;
  const uint64_t ts = (t + 3ull * (uint64_t)n / 2) % m2;
  Q2 r;
  r.re = cosq(M_PIq * (__float128)t / (__float128)n);
  r.im = cosq(M_PIq * (__float128)ts / (__float128)n);
  return r;
}

// a slot map out[p] = sum_d A[d][p] in[(p + d) mod S], offsets d in [0, S)
using DiagMap = std::map<int, std::vector<Q2>>;

// one stage on ns slots (ns = N/2, or the sparse n): the n-slot FFT's twiddles
// are the N/2-slot FFT's, zeta^((N/2m) 5^j)
DiagMap stage(int n, int ns, int m, bool inverse) {
  const int S = ns, h = m / 2;
  const uint64_t m2 = 2ull * (uint64_t)n;
  DiagMap A;
  auto at = [&](int d) -> std::vector<Q2>& {
    auto it = A.find(d);
    if (it == A.end()) it = A.emplace(d, std::vector<Q2>(S)).first;
    return it->second;
  };
  // D_m[j] = zeta^((N/2m) 5^j), j < m/2
  std::vector<Q2> D_m(h);
  uint64_t g5 = 1;
  for (int j = 0; j < h; ++j) {
    D_m[j] = root((uint64_t)(n / 2 / m) * g5, n);
    g5 = g5 * 5 % m2;
  }
  for (int p = 0; p < S; ++p) {
    const int r = p % m;
    const int j = r < h ? r : r - h;
    const Q2& D = D_m[j];
    if (!inverse) {
      if (r < h) {
        at(0)[p] = Q2{1, 0};
        at(h % S)[p] = D;
      } else {
        at(0)[p] = Q2{-D.re, -D.im};
        at((S - h) % S)[p] = Q2{1, 0};
      }
    } else {
      const __float128 half = 0.5Q;
      if (r < h) {
        at(0)[p] = Q2{half, 0};
        at(h % S)[p] = Q2{half, 0};
      } else {
        const Q2 Dc{D.re * half, -D.im * half};
        at((S - h) % S)[p] = Dc;
        at(0)[p] = Q2{-Dc.re, -Dc.im};
      }
    }
  }
  return A;
}

// (A B): B applied first; (AB)[d1 + d2][p] += A[d1][p] B[d2][p + d1]
DiagMap compose(const DiagMap& A, const DiagMap& B, int S) {
  DiagMap R;
  for (const auto& a : A) {
    for (const auto& b : B) {
      const int d = (a.first + b.first) % S;
      auto it = R.find(d);
      if (it == R.end()) it = R.emplace(d, std::vector<Q2>(S)).first;
      std::vector<Q2>& out = it->second;
      for (int p = 0; p < S; ++p) {
        const Q2& x = a.second[p];
        if (qzero(x)) continue;
        const Q2 t = qmul(x, b.second[(p + a.first) % S]);
        out[p].re += t.re;
        out[p].im += t.im;
      }
    }
  }
  return R;
}

}  // namespace

int boot_group_len(int log_slots, int groups, int g) { return log_slots / groups + (g < log_slots % groups ? 1 : 0); }

// The sparse transforms differ from the n-slot maps in two groups: the last
// CoeffToSlot group writes [w, 0] with period 2n (the n-slot diagonal on the
// lower half of each period, zero on the upper), and the first SlotToCoeff
// group reads [a, b] with period 2n and transforms a + i b.
static bool widened(int log_n, int log_ns, int groups, int inverse, int g) {
  return log_ns < log_n - 1 && (inverse ? g == groups - 1 : g == 0);
}

BootGroupTable boot_group_geometry(int log_n, int log_ns, int groups, int inverse, int g) {
  const int S = 1 << log_ns, L = log_ns;
  int first = 0;
  for (int i = 0; i < g; ++i) first += boot_group_len(L, groups, i);
  BootGroupTable t;
  t.len = boot_group_len(L, groups, g);
  int mmin = S;
  for (int i = 0; i < t.len; ++i) {
    const int idx = first + i;
    const int m = inverse ? 1 << (L - idx) : 1 << (idx + 1);
    if (m < mmin) mmin = m;
  }
  t.ns = widened(log_n, log_ns, groups, inverse, g) ? 2 * S : S;
  t.delta = mmin / 2;
  t.E = t.ns / t.delta;
  t.n1 = 1 << ((t.len + 2) / 2);
  if (t.n1 > S / t.delta) t.n1 = S / t.delta;
  return t;
}

BootGroupTable boot_group_table(int log_n, int log_ns, int groups, int K, int ratio, int inverse, int g) {
  const int n = 1 << log_n, S = 1 << log_ns, L = log_ns;
  BootGroupTable t = boot_group_geometry(log_n, log_ns, groups, inverse, g);
  int first = 0;
  for (int i = 0; i < g; ++i) first += boot_group_len(L, groups, i);
  DiagMap M;
  for (int i = 0; i < t.len; ++i) {
    const int idx = first + i;
    const int m = inverse ? 1 << (L - idx) : 1 << (idx + 1);
    DiagMap st = stage(n, S, m, inverse != 0);
    M = i == 0 ? st : compose(st, M, S);
  }
  if (g == 0) {
    // CoeffToSlot: 1 / (2 (K+1)) (the real/imaginary split doubles, EvalMod
    // reads x / (K+1)), and for the sparse transform n / (N/2) against the
    // trace's factor N/2n; SlotToCoeff: 2^ratio / (2 pi) (back from sin(2 pi x))
    __float128 k = inverse ? 1.0Q / (2.0Q * (__float128)(K + 1)) : ldexpq(1.0Q, ratio) / (2.0Q * M_PIq);
    if (inverse) k = k * (__float128)S / (__float128)(n / 2);
    for (auto& d : M)
      for (Q2& v : d.second) {
        v.re *= k;
        v.im *= k;
      }
  }
  if (t.ns != S) {
    const int S2 = t.ns;
    DiagMap W;
    for (const auto& d : M) {
      if (inverse) {
        // an n-periodic input reads the same slot at d and d - n: keep the
        // centred offset; zero on the upper half of each 2n period
        std::vector<Q2> v(S2);
        for (int p = 0; p < S; ++p) v[p] = d.second[p];
        W[d.first < S / 2 ? d.first : d.first + S] = std::move(v);
      } else {
        // offsets d and d + n; a slot read from the upper half is times i
        for (int k = 0; k < 2; ++k) {
          const int off = (d.first + k * S) % S2;
          auto it = W.find(off);
          if (it == W.end()) it = W.emplace(off, std::vector<Q2>(S2)).first;
          for (int p = 0; p < S2; ++p) {
            const Q2& v = d.second[p % S];
            const bool upper = (p + off) % S2 >= S;
            it->second[p].re += upper ? -v.im : v.re;
            it->second[p].im += upper ? v.re : v.im;
          }
        }
      }
    }
    M.swap(W);
  }
  for (const auto& d : M) {
    BootDiag bd;
    bd.off = d.first;
    bd.re.resize(t.ns);
    bd.im.resize(t.ns);
    for (int p = 0; p < t.ns; ++p) {
      bd.re[p] = (double)d.second[p].re;
      bd.im[p] = (double)d.second[p].im;
    }
    t.diags.push_back(std::move(bd));
  }
  return t;
}

void boot_cheb_coeffs(int K, int r, int deg, double* out) {
  const int n = deg + 1;
  std::vector<__float128> fk(n), th(n);
  for (int k = 0; k < n; ++k) {
    th[k] = M_PIq * ((__float128)k + 0.5Q) / (__float128)n;
    const __float128 u = cosq(th[k]);
    fk[k] = cosq(2.0Q * M_PIq * ((__float128)(K + 1) * u - 0.25Q) / ldexpq(1.0Q, r));
  }
  for (int j = 0; j <= deg; ++j) {
    __float128 s = 0;
    for (int k = 0; k < n; ++k) s += fk[k] * cosq((__float128)j * th[k]);
    s = s * 2.0Q / (__float128)n;
    if (j == 0) s = s / 2;
    out[j] = (double)s;
  }
}

}  // namespace secpe
