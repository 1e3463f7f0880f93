// HIP kernels for RNS-CKKS on gfx950 (CDNA4, wave64).
//
// All kernels are batched through job descriptors (jobs.h) and use the exact
// binary64 modular arithmetic of modarith.h.  Polynomials live in HBM limb by
// limb (limb-major), each limb N canonical residues.
//
// Paper: arXiv 2502.00847, Sec. 2.2 (RNS-CKKS over Z_Q[X]/(X^N+1), the
// homomorphic add / mult / rotate the Argmax is built from).
#include "kernels.h"

namespace secpe {

// largest key-switch digit (alpha primes) and special-prime count
constexpr int MAX_DIGIT = 16;

// ---------------------------------------------------------------------------
// negacyclic NTT
//
// Forward: merged Cooley-Tukey (natural order in, bit-reversed evaluation order
// out): stage g pairs j and j + N/2^(g+1) with twiddle psi^bitrev(2^g + i),
// i = j >> (logN - g).  Inverse: the Gentleman-Sande mirror with psi^-1, then
// the factor N^-1.  For N > 2^12 the transform is split in two passes over a
// 2^k1 x 2^k2 view of the limb: the first k1 stages only mix elements of one
// column (stride 2^k2), the last k2 stages only elements of one row.  Each
// workgroup stages a 4096-element tile in LDS; each round keeps up to 16
// elements in registers and runs up to four radix-2 stages on them.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int lpad(int i) { return i + (i >> 4); }

// Pair p (elements 2p, 2p+1) of a G x S tile taken by the calling thread in its
// slot q < G*S/512.  With rows of S = 256, the row-pass thread maps give each
// wave four whole rows (16 lanes per row), and this map keeps a wave's pairs
// inside those rows too: the tile's LDS traffic then never crosses waves, and
// tile_sync orders it within the wave instead of across the workgroup.
template <int S>
__device__ __forceinline__ int tile_pair(int q) {
  const int t = threadIdx.x;
  return S == 256 ? (t >> 6) * 512 + q * 64 + (t & 63) : t + 256 * q;
}
template <int S>
__device__ __forceinline__ void tile_sync() {
  if (S == 256) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  } else {
    __syncthreads();
  }
}

// canonical residue, or centred in (-p/2, p/2] (the digits of a centred base conversion)
__device__ __forceinline__ double canon_out(double v, const Mod& m, int centre) {
  const double c = canon(v, m);
  return centre && 2.0 * c > m.p ? c - m.p : c;
}

__device__ __forceinline__ double2 ld2(const double* p, size_t o) {
  const dv2 v = *(cgdbl2*)(CGPTR(p) + o);
  return make_double2(v.x, v.y);
}
__device__ __forceinline__ void st2(double* p, size_t o, double a, double b) {
  dv2 v;
  v.x = a;
  v.y = b;
  *(gdbl2*)(GPTR(p) + o) = v;
}

// fused prologue: residue z mod q_src taken centred, reduced mod m
__device__ __forceinline__ double spread_in(double z, double q_src, const Mod& m) {
  return red(2.0 * z > q_src ? z - q_src : z, m);
}

// fused epilogue of a forward transform: v0, v1 are the (lazily reduced)
// transform values at positions o, o + 1 of limb l
__device__ __forceinline__ void ntt_epilogue(const NttJob& J, int l, size_t o, double v0, double v1, const Mod& m) {
  const double c0 = canon(v0, m), c1 = canon(v1, m);
  const double k = KPTR(J.ek)[l];
  double r0, r1;
  if (J.epi == EPI_RESCALE) {
    const double2 a = ld2(J.ea, o);
    r0 = mul_mod(a.x - c0, k, m);
    r1 = mul_mod(a.y - c1, k, m);
  } else if (J.epi == EPI_LINRS) {
    const double2 a = ld2(J.ea, o);
    const double2 b = J.eb ? ld2(J.eb, o) : make_double2(0.0, 0.0);
    const double ka = KPTR(J.ek2)[l];
    double sx = mul_mod(a.x, ka, m), sy = mul_mod(a.y, ka, m);
    if (J.eb) {
      const double kb = KPTR(J.ek3)[l];
      sx += mul_mod(b.x, kb, m);
      sy += mul_mod(b.y, kb, m);
    }
    r0 = mul_mod(canon(sx, m) - c0, k, m);
    r1 = mul_mod(canon(sy, m) - c1, k, m);
  } else if (J.epi == EPI_RRCOMB) {
    const double k2 = KPTR(J.ek2)[l];
    double2 a = ld2(J.ea, o);
    const double2 b = ld2(J.eb, o);
    if (J.sq == 1) {
      a.x = mul_mod(a.x, a.x, m);
      a.y = mul_mod(a.y, a.y, m);
    } else if (J.sq == 2) {
      const double2 a1 = ld2(J.ebase, o);
      a.x = mul_mod(2.0 * a.x, a1.x, m);
      a.y = mul_mod(2.0 * a.y, a1.y, m);
    }
    r0 = mul_mod(red(mul_mod(a.x, k2, m) + (b.x - c0), m), k, m);
    r1 = mul_mod(red(mul_mod(a.y, k2, m) + (b.y - c1), m), k, m);
  } else {
    const double2 b = ld2(J.eb, o);
    r0 = mul_mod(b.x - c0, k, m);
    r1 = mul_mod(b.y - c1, k, m);
    if (J.ebase) {
      const double2 base = ld2(J.ebase, o);
      r0 += base.x;
      r1 += base.y;
    }
  }
  st2(J.eout, o, canon(r0, m), canon(r1, m));
}

// The same epilogue over a row tile held in LDS (lazily reduced values at
// lpad(2i), lpad(2i+1) for pair i = tile_pair(q), q < NPP, pair i at offset
// o0 + 2i of limb l).  Pairs go in batches of NB: every operand of a batch is
// requested at once, so a batch costs one load round trip, not one per pair.
template <int NPP, int S>
__device__ __forceinline__ void row_epilogue(const NttJob& J, int l, size_t o0, const double* lds, const Mod& m) {
  constexpr int NB = NPP / 2;
  const double k = KPTR(J.ek)[l];
  const double k2 = J.epi == EPI_RRCOMB ? KPTR(J.ek2)[l] : 0.0;
#pragma unroll
  for (int h = 0; h < NPP / NB; ++h) {
    auto off = [&](int r) -> size_t { return o0 + 2 * (size_t)tile_pair<S>(h * NB + r); };
    auto val = [&](int r, int c) -> double { return canon(lds[lpad(2 * tile_pair<S>(h * NB + r) + c)], m); };
    dv2 a[NB], b[NB];
    if (J.epi == EPI_RESCALE) {
#pragma unroll
      for (int r = 0; r < NB; ++r) a[r] = *(cgdbl2*)(CGPTR(J.ea) + off(r));
#pragma unroll
      for (int r = 0; r < NB; ++r) {
        const double r0 = mul_mod(a[r].x - val(r, 0), k, m);
        const double r1 = mul_mod(a[r].y - val(r, 1), k, m);
        st2(J.eout, off(r), canon(r0, m), canon(r1, m));
      }
    } else if (J.epi == EPI_LINRS) {
      const double ka = KPTR(J.ek2)[l];
      const double kb = J.eb ? KPTR(J.ek3)[l] : 0.0;
#pragma unroll
      for (int r = 0; r < NB; ++r) a[r] = *(cgdbl2*)(CGPTR(J.ea) + off(r));
      if (J.eb) {
#pragma unroll
        for (int r = 0; r < NB; ++r) b[r] = *(cgdbl2*)(CGPTR(J.eb) + off(r));
      }
#pragma unroll
      for (int r = 0; r < NB; ++r) {
        double sx = mul_mod(a[r].x, ka, m), sy = mul_mod(a[r].y, ka, m);
        if (J.eb) {
          sx += mul_mod(b[r].x, kb, m);
          sy += mul_mod(b[r].y, kb, m);
        }
        const double r0 = mul_mod(canon(sx, m) - val(r, 0), k, m);
        const double r1 = mul_mod(canon(sy, m) - val(r, 1), k, m);
        st2(J.eout, off(r), canon(r0, m), canon(r1, m));
      }
    } else if (J.epi == EPI_RRCOMB) {
#pragma unroll
      for (int r = 0; r < NB; ++r) {
        a[r] = *(cgdbl2*)(CGPTR(J.ea) + off(r));
        b[r] = *(cgdbl2*)(CGPTR(J.eb) + off(r));
      }
      if (J.sq == 1) {
#pragma unroll
        for (int r = 0; r < NB; ++r) {
          a[r].x = mul_mod(a[r].x, a[r].x, m);
          a[r].y = mul_mod(a[r].y, a[r].y, m);
        }
      } else if (J.sq == 2) {
        dv2 a1[NB];
#pragma unroll
        for (int r = 0; r < NB; ++r) a1[r] = *(cgdbl2*)(CGPTR(J.ebase) + off(r));
#pragma unroll
        for (int r = 0; r < NB; ++r) {
          a[r].x = mul_mod(2.0 * a[r].x, a1[r].x, m);
          a[r].y = mul_mod(2.0 * a[r].y, a1[r].y, m);
        }
      }
#pragma unroll
      for (int r = 0; r < NB; ++r) {
        const double r0 = mul_mod(red(mul_mod(a[r].x, k2, m) + (b[r].x - val(r, 0)), m), k, m);
        const double r1 = mul_mod(red(mul_mod(a[r].y, k2, m) + (b[r].y - val(r, 1)), m), k, m);
        st2(J.eout, off(r), canon(r0, m), canon(r1, m));
      }
    } else {
#pragma unroll
      for (int r = 0; r < NB; ++r) b[r] = *(cgdbl2*)(CGPTR(J.eb) + off(r));
      if (J.ebase) {
#pragma unroll
        for (int r = 0; r < NB; ++r) a[r] = *(cgdbl2*)(CGPTR(J.ebase) + off(r));
      }
#pragma unroll
      for (int r = 0; r < NB; ++r) {
        double r0 = mul_mod(b[r].x - val(r, 0), k, m);
        double r1 = mul_mod(b[r].y - val(r, 1), k, m);
        if (J.ebase) {
          r0 += a[r].x;
          r1 += a[r].y;
        }
        st2(J.eout, off(r), canon(r0, m), canon(r1, m));
      }
    }
  }
}

enum { NTT_SINGLE = 0, NTT_COL = 1, NTT_ROW = 2 };

template <int LOGS, int MODE>
__device__ __forceinline__ int tw_index(int u, int v, int row, int k1) {
  int idx = (1 << u) + (v >> (LOGS - u));
  if (MODE == NTT_ROW) idx = (1 << (k1 + u)) + (row << u) + (v >> (LOGS - u));
  return idx;
}

template <int LOGS, int G, int R, int MODE>
__device__ __forceinline__ void fwd_round(double* lds, int u0, const double* __restrict__ tw,
                                          const double* __restrict__ twq, const Mod& m, int row0, int k1) {
  constexpr int S = 1 << LOGS;
  constexpr int NG = (G * S) >> R;
  const int b_hi = LOGS - 1 - u0;
  const int b_lo = LOGS - u0 - R;
  for (int grp = threadIdx.x; grp < NG; grp += blockDim.x) {
    const int vec = grp / (S >> R);
    const int rem = grp % (S >> R);
    const int low = rem & ((1 << b_lo) - 1);
    const int high = rem >> b_lo;
    const int base = (high << (b_hi + 1)) | low;
    double x[1 << R];
#pragma unroll
    for (int e = 0; e < (1 << R); ++e) x[e] = lds[lpad(vec * S + (base | (e << b_lo)))];
#pragma unroll
    for (int w = 0; w < R; ++w) {
      const int u = u0 + w;
      const int half = 1 << (R - 1 - w);
#pragma unroll
      for (int e0 = 0; e0 < (1 << R); ++e0) {
        if (e0 & half) continue;
        const int e1 = e0 + half;
        const int v = base | (e0 << b_lo);
        const int idx = tw_index<LOGS, MODE>(u, v, row0 + vec, k1);
        const double U = red(x[e0], m);
        const double T = mul_w(x[e1], tw[idx], twq[idx], m.p);
        x[e0] = U + T;
        x[e1] = U - T;
      }
    }
#pragma unroll
    for (int e = 0; e < (1 << R); ++e) lds[lpad(vec * S + (base | (e << b_lo)))] = x[e];
  }
}

template <int LOGS, int G, int R, int MODE>
__device__ __forceinline__ void inv_round(double* lds, int b_lo, const double* __restrict__ tw,
                                          const double* __restrict__ twq, const Mod& m, int row0, int k1) {
  constexpr int S = 1 << LOGS;
  constexpr int NG = (G * S) >> R;
  const int b_hi = b_lo + R - 1;
  for (int grp = threadIdx.x; grp < NG; grp += blockDim.x) {
    const int vec = grp / (S >> R);
    const int rem = grp % (S >> R);
    const int low = rem & ((1 << b_lo) - 1);
    const int high = rem >> b_lo;
    const int base = (high << (b_hi + 1)) | low;
    double x[1 << R];
#pragma unroll
    for (int e = 0; e < (1 << R); ++e) x[e] = lds[lpad(vec * S + (base | (e << b_lo)))];
#pragma unroll
    for (int w = 0; w < R; ++w) {
      const int u = LOGS - 1 - (b_lo + w);
      const int half = 1 << w;
#pragma unroll
      for (int e0 = 0; e0 < (1 << R); ++e0) {
        if (e0 & half) continue;
        const int e1 = e0 + half;
        const int v = base | (e0 << b_lo);
        const int idx = tw_index<LOGS, MODE>(u, v, row0 + vec, k1);
        const double U = red(x[e0], m);
        const double V = red(x[e1], m);
        x[e0] = U + V;
        x[e1] = mul_w(U - V, tw[idx], twq[idx], m.p);
      }
    }
#pragma unroll
    for (int e = 0; e < (1 << R); ++e) lds[lpad(vec * S + (base | (e << b_lo)))] = x[e];
  }
}

template <int LOGS, int G, int MODE, int U0>
__device__ __forceinline__ void fwd_all(double* lds, const double* tw, const double* twq, const Mod& m, int row0, int k1) {
  if constexpr (U0 < LOGS) {
    constexpr int R = (LOGS - U0) < 4 ? (LOGS - U0) : 4;
    fwd_round<LOGS, G, R, MODE>(lds, U0, tw, twq, m, row0, k1);
    __syncthreads();
    fwd_all<LOGS, G, MODE, U0 + R>(lds, tw, twq, m, row0, k1);
  }
}

template <int LOGS, int G, int MODE, int B0>
__device__ __forceinline__ void inv_all(double* lds, const double* tw, const double* twq, const Mod& m, int row0, int k1) {
  if constexpr (B0 < LOGS) {
    constexpr int R = (LOGS - B0) < 4 ? (LOGS - B0) : 4;
    inv_round<LOGS, G, R, MODE>(lds, B0, tw, twq, m, row0, k1);
    __syncthreads();
    inv_all<LOGS, G, MODE, B0 + R>(lds, tw, twq, m, row0, k1);
  }
}

template <int LOGS, int G, int MODE, bool INV>
__global__ __launch_bounds__(256) void k_ntt(const NttJob* __restrict__ jobs, DevTables T, int second) {
  extern __shared__ double lds[];
  const NttJob J = jobs[blockIdx.y];
  const int l = blockIdx.z;
  if (l >= J.n_limbs || (l >= J.skip_lo && l < J.skip_hi)) return;
  const int pr = l < J.n_chain ? l : T.n_q + (l - J.n_chain);
  const int log_n = T.log_n;
  const int N = 1 << log_n;
  constexpr int S = 1 << LOGS;
  const Mod m{KPTR(T.mod)[pr], KPTR(T.minv)[pr]};
  const double* tw = (INV ? T.ipsi : T.psi) + (size_t)pr * N;
  const double* twq = (INV ? T.ipsiq : T.psiq) + (size_t)pr * N;
  const bool spread = !INV && !second && J.spread_from > 0;
  const double* src = (second ? J.dst : J.src) + (spread ? 0 : (size_t)l * N);
  const double q_src = spread ? KPTR(T.mod)[J.spread_from - 1] : 0.0;
  double* dst = J.dst + (size_t)l * N;
  const int tid = threadIdx.x;
  const int k1 = log_n - LOGS;
  const int C = N >> LOGS;            // number of vectors of length S
  int row0 = 0;
  if (MODE == NTT_COL) {
    const int c0 = blockIdx.x * G;
    for (int i = tid; i < G * S / 2; i += blockDim.x) {
      const int cp = i % (G / 2);
      const int v = i / (G / 2);
      const double2 val = *reinterpret_cast<const double2*>(src + (size_t)v * C + c0 + 2 * cp);
      lds[lpad((2 * cp) * S + v)] = val.x;
      lds[lpad((2 * cp + 1) * S + v)] = val.y;
    }
  } else {
    row0 = blockIdx.x * G;
    const double2* s2 = reinterpret_cast<const double2*>(src + (size_t)row0 * S);
    for (int i = tid; i < G * S / 2; i += blockDim.x) {
      const double2 val = s2[i];
      lds[lpad(2 * i)] = spread ? spread_in(val.x, q_src, m) : val.x;
      lds[lpad(2 * i + 1)] = spread ? spread_in(val.y, q_src, m) : val.y;
    }
  }
  __syncthreads();
  if (INV) inv_all<LOGS, G, MODE, 0>(lds, tw, twq, m, row0, k1);
  else fwd_all<LOGS, G, MODE, 0>(lds, tw, twq, m, row0, k1);
  const bool scale = INV && MODE != NTT_ROW;
  const double ni = T.ninv[pr], niq = T.ninvq[pr];
  if (MODE == NTT_COL) {
    const int c0 = blockIdx.x * G;
    for (int i = tid; i < G * S / 2; i += blockDim.x) {
      const int cp = i % (G / 2);
      const int v = i / (G / 2);
      double a = lds[lpad((2 * cp) * S + v)];
      double b = lds[lpad((2 * cp + 1) * S + v)];
      if (scale) { a = mul_w(red(a, m), ni, niq, m.p); b = mul_w(red(b, m), ni, niq, m.p); }
      *reinterpret_cast<double2*>(dst + (size_t)v * C + c0 + 2 * cp) = make_double2(canon(a, m), canon(b, m));
    }
  } else {
    double2* d2 = reinterpret_cast<double2*>(dst + (size_t)row0 * S);
    const bool epi = !INV && MODE != NTT_COL && J.epi != EPI_NONE;
    for (int i = tid; i < G * S / 2; i += blockDim.x) {
      double a = lds[lpad(2 * i)];
      double b = lds[lpad(2 * i + 1)];
      if (scale && J.ek) {
        const double ys = KPTR(J.ek)[l];
        a = mul_mod(red(a, m), ys, m);
        b = mul_mod(red(b, m), ys, m);
      } else if (scale) {
        a = mul_w(red(a, m), ni, niq, m.p);
        b = mul_w(red(b, m), ni, niq, m.p);
      }
      if (epi) ntt_epilogue(J, l, (size_t)l * N + (size_t)row0 * S + 2 * i, a, b, m);
      else d2[i] = make_double2(canon_out(a, m, J.centre), canon_out(b, m, J.centre));
    }
  }
}

// ---------------------------------------------------------------------------
// two-pass transform for N = 2^13 .. 2^16.  A workgroup owns G vectors of
// S = 2^LOGS elements (G*S = 4096).  Round A runs the four stages on the top
// four bits of the vector index, round B the remaining LOGS-4 stages; each
// thread keeps its elements in registers for a round, and LDS is only used to
// move between the two rounds' layouts.  Thread maps are chosen so that every
// global access of a wavefront is made of 128-byte runs:
//   column pass (elements v*C + c of columns c0..c0+G-1): lanes run over c;
//   row pass (contiguous rows of S): lanes run over consecutive elements,
//   with an LDS transpose for the round whose thread owns a contiguous run.
// ---------------------------------------------------------------------------
// One round of R radix-2 stages on x[0 .. 2^R): element e sits at vector
// position v = (vhigh << (b_lo + R)) | (e << b_lo) | low.  The twiddle of a
// stage depends only on the bits of v above the butterfly's bit, so a stage
// needs 2^(R - 1 - eb) distinct twiddles (eb = butterfly bit within e); they
// are fetched once per stage (wave-uniform in the column pass's first round).
template <int LOGS, int R, int MODE, bool INV>
__device__ __forceinline__ void ntt_round(double* x, int vhigh, int b_lo, int row, int k1, kdbl* __restrict__ tw,
                                          kdbl* __restrict__ twq, const Mod& m) {
#pragma unroll
  for (int w = 0; w < R; ++w) {
    // forward: highest bit first; inverse: lowest bit first
    const int eb = INV ? w : (R - 1 - w);
    const int half = 1 << eb;
    const int u = LOGS - 1 - (b_lo + eb);
    const int nt = 1 << (R - 1 - eb);
    // v >> (LOGS - u) = (vhigh << (R - 1 - eb)) | (e0 >> (eb + 1))
    int base = (MODE == NTT_ROW) ? (1 << (k1 + u)) + (row << u) : (1 << u);
    base += vhigh << (R - 1 - eb);
    double wv[1 << (R - 1)], wq[1 << (R - 1)];
#pragma unroll
    for (int j = 0; j < (1 << (R - 1)); ++j) {
      if (j < nt) {
        wv[j] = tw[base + j];
        wq[j] = twq[base + j];
      }
    }
#pragma unroll
    for (int e0 = 0; e0 < (1 << R); ++e0) {
      if (e0 & half) continue;
      const int e1 = e0 + half;
      const int j = e0 >> (eb + 1);
      if (!INV) {
        const double U = red(x[e0], m);
        const double T = mul_w(x[e1], wv[j], wq[j], m.p);
        x[e0] = U + T;
        x[e1] = U - T;
      } else {
        const double U = red(x[e0], m);
        const double V = red(x[e1], m);
        x[e0] = U + V;
        x[e1] = mul_w(U - V, wv[j], wq[j], m.p);
      }
    }
  }
}

// Forward column pass from registers: x[e] holds element v = e*NB + la of
// column va = t % G (la = t / G) of the tile whose first column is c0; runs
// rounds A and B and stores the column-passed tile to dst (one limb).
template <int LOGS, int G>
__device__ __forceinline__ void fwd_col_from_regs(double* x, double* lds, gdbl* dst, int c0, int k1, kdbl* tw,
                                                  kdbl* twq, const Mod& m) {
  constexpr int S = 1 << LOGS;
  constexpr int RB = LOGS - 4;
  constexpr int NB = 1 << RB;
  constexpr int GB = 16 / NB;
  const int t = threadIdx.x;
  const int C = (1 << (k1 + LOGS)) >> LOGS;
  const int va = t % G, la = t / G;
  ntt_round<LOGS, 4, NTT_COL, false>(x, 0, RB, va, k1, tw, twq, m);
#pragma unroll
  for (int e = 0; e < 16; ++e) lds[va * (S + 1) + e * NB + la] = x[e];
  __syncthreads();
#pragma unroll
  for (int gi = 0; gi < GB; ++gi) {
    const int grp = t + gi * 256;
    const int vb = grp % G, hb = grp / G;
    double y[NB];
#pragma unroll
    for (int e = 0; e < NB; ++e) y[e] = lds[vb * (S + 1) + hb * NB + e];
    ntt_round<LOGS, RB, NTT_COL, false>(y, hb, 0, vb, k1, tw, twq, m);
#pragma unroll
    for (int e = 0; e < NB; ++e) dst[(size_t)(hb * NB + e) * C + c0 + vb] = canon(y[e], m);
  }
}

// Inverse row pass (the first pass of the inverse transform) on one G x S
// tile already in LDS in row layout (element e of row v at lpad(v*S + e)):
// rounds B and A, then the tile is stored canonically to rows row0 .. of dst
// (one limb; no N^-1, which the column pass applies).
template <int LOGS, int G>
__device__ __forceinline__ void inv_row_from_lds(double* lds, gdbl* dst, int row0, int k1, kdbl* tw, kdbl* twq,
                                                 const Mod& m) {
  constexpr int S = 1 << LOGS;
  constexpr int RB = LOGS - 4;
  constexpr int NB = 1 << RB;
  constexpr int GB = 16 / NB;
  const int t = threadIdx.x;
#pragma unroll
  for (int gi = 0; gi < GB; ++gi) {
    const int grp = t + gi * 256;
    const int vb = grp / 16, hb = grp % 16;
    double y[NB];
#pragma unroll
    for (int e = 0; e < NB; ++e) y[e] = lds[lpad(vb * S + hb * NB + e)];
    ntt_round<LOGS, RB, NTT_ROW, true>(y, hb, 0, row0 + vb, k1, tw, twq, m);
    // each group is read and written back by its own thread: no barrier needed here
#pragma unroll
    for (int e = 0; e < NB; ++e) lds[lpad(vb * S + hb * NB + e)] = y[e];
  }
  tile_sync<S>();
  const int va = t / NB, la = t % NB;
  double x[16];
#pragma unroll
  for (int e = 0; e < 16; ++e) x[e] = lds[lpad(va * S + e * NB + la)];
  ntt_round<LOGS, 4, NTT_ROW, true>(x, 0, RB, row0 + va, k1, tw, twq, m);
#pragma unroll
  for (int e = 0; e < 16; ++e) dst[(size_t)(row0 + va) * S + e * NB + la] = canon(x[e], m);
}

// The row passes are compiled for the 4 waves per SIMD that their 34 KiB LDS
// tile allows (the compiler cannot see the dynamic LDS size and would
// otherwise keep registers low for 8 and not hoist the twiddle loads); the
// column passes measure best at the compiler's default.
// P (column passes): tiles per workgroup; the loads of all P tiles are
// issued before the first is transformed, so that the later tiles' loads are
// in flight while the earlier ones compute.
template <int LOGS, int G, int MODE, bool INV, int P>
__global__ __launch_bounds__(256)
__attribute__((amdgpu_waves_per_eu(MODE == NTT_ROW ? (P == 1 ? 4 : 2) : 1, MODE == NTT_ROW ? 4 : 8))) void k_ntt2(const NttJob* __restrict__ jobs, DevTables T, int second) {
  extern __shared__ double lds[];
  constexpr int S = 1 << LOGS;
  constexpr int RB = LOGS - 4;         // bits of round B
  constexpr int NB = 1 << RB;          // elements per round-B group
  constexpr int GB = 16 / NB;          // round-B groups per thread
  const NttJob J = jobs[blockIdx.y];
  const int l = blockIdx.z;
  if (l >= J.n_limbs || (l >= J.skip_lo && l < J.skip_hi)) return;
  const int pr = l < J.n_chain ? l : T.n_q + (l - J.n_chain);
  const int log_n = T.log_n;
  const int N = 1 << log_n;
  const Mod m{KPTR(T.mod)[pr], KPTR(T.minv)[pr]};
  kdbl* tw = KPTR(INV ? T.ipsi : T.psi) + (size_t)pr * N;
  kdbl* twq = KPTR(INV ? T.ipsiq : T.psiq) + (size_t)pr * N;
  const bool spread = !INV && MODE == NTT_COL && J.spread_from > 0;
  cgdbl* src = CGPTR(second ? J.dst : J.src) + (spread ? 0 : (size_t)l * N);
  const double q_src = spread ? KPTR(T.mod)[J.spread_from - 1] : 0.0;
  gdbl* dst = GPTR(J.dst) + (size_t)l * N;
  const int t = threadIdx.x;
  const int k1 = log_n - LOGS;
  const int C = N >> LOGS;
  const bool scale = INV && MODE == NTT_COL;
  const double ni = KPTR(T.ninv)[pr], niq = KPTR(T.ninvq)[pr];
  // round-A ownership: vector va, low part la; elements v = e*NB + la, e < 16
  const int va = MODE == NTT_COL ? (t % G) : (t / NB);
  const int la = MODE == NTT_COL ? (t / G) : (t % NB);
  const int c0 = MODE == NTT_COL ? blockIdx.x * G : 0;
  const int row0 = MODE == NTT_ROW ? blockIdx.x * G : 0;
  double x[16];
  auto gaddr = [&](int vec, int v) -> size_t {
    return MODE == NTT_COL ? (size_t)v * C + c0 + vec : (size_t)(row0 + vec) * S + v;
  };
  // LDS index: the column pass pads one element per vector (lanes run over
  // vectors), the row pass one per 16 elements (lanes run within a vector)
  auto lidx = [&](int vec, int v) -> int { return MODE == NTT_COL ? vec * (S + 1) + v : lpad(vec * S + v); };
  if (!INV && MODE == NTT_COL) {
    if constexpr (P == 1) {
#pragma unroll
    for (int e = 0; e < 16; ++e) x[e] = src[gaddr(va, e * NB + la)];
    if (spread) {
#pragma unroll
      for (int e = 0; e < 16; ++e) x[e] = spread_in(x[e], q_src, m);
    }
    fwd_col_from_regs<LOGS, G>(x, lds, dst, c0, k1, tw, twq, m);
    } else {
    double xs[P][16];
#pragma unroll
    for (int p = 0; p < P; ++p) {
      const int cp = (blockIdx.x * P + p) * G;
#pragma unroll
      for (int e = 0; e < 16; ++e) xs[p][e] = src[(size_t)(e * NB + la) * C + cp + va];
    }
#pragma unroll
    for (int p = 0; p < P; ++p) {
      if (spread) {
#pragma unroll
        for (int e = 0; e < 16; ++e) xs[p][e] = spread_in(xs[p][e], q_src, m);
      }
      if (p) __syncthreads();   // the tile in LDS is read by every thread before it is reused
      fwd_col_from_regs<LOGS, G>(xs[p], lds, dst, (blockIdx.x * P + p) * G, k1, tw, twq, m);
    }
    }
  } else if (!INV) {
    if constexpr (P == 1) {
    // ---- round A straight from global memory
#pragma unroll
    for (int e = 0; e < 16; ++e) x[e] = src[gaddr(va, e * NB + la)];
    ntt_round<LOGS, 4, MODE, false>(x, 0, RB, row0 + va, k1, tw, twq, m);
#pragma unroll
    for (int e = 0; e < 16; ++e) lds[lidx(va, e * NB + la)] = x[e];
    // (this branch is the row pass: the exchange stays inside each wave at S = 256)
    tile_sync<S>();
    // ---- round B
#pragma unroll
    for (int gi = 0; gi < GB; ++gi) {
      const int grp = t + gi * 256;
      const int vb = MODE == NTT_COL ? (grp % G) : (grp / 16);
      const int hb = MODE == NTT_COL ? (grp / G) : (grp % 16);
      double y[NB];
#pragma unroll
      for (int e = 0; e < NB; ++e) y[e] = lds[lidx(vb, hb * NB + e)];
      ntt_round<LOGS, RB, MODE, false>(y, hb, 0, row0 + vb, k1, tw, twq, m);
      if (MODE == NTT_COL) {
#pragma unroll
        for (int e = 0; e < NB; ++e) dst[gaddr(vb, hb * NB + e)] = canon(y[e], m);
      } else {
#pragma unroll
        for (int e = 0; e < NB; ++e) lds[lidx(vb, hb * NB + e)] = y[e];
      }
    }
    if (MODE == NTT_ROW) {
      tile_sync<S>();
      if (J.epi != EPI_NONE) {
        row_epilogue<G * S / 2 / 256, S>(J, l, (size_t)l * N + (size_t)row0 * S, lds, m);
      } else {
        gdbl2* d2 = (gdbl2*)(dst + (size_t)row0 * S);
#pragma unroll
        for (int q = 0; q < G * S / 2 / 256; ++q) {
          const int i = tile_pair<S>(q);
          dv2 v;
          v.x = canon(lds[lpad(2 * i)], m);
          v.y = canon(lds[lpad(2 * i + 1)], m);
          d2[i] = v;
        }
      }
    }
    } else {
    // (the forward row pass; P tiles of rows, every tile's loads issued first)
    double xs[P][16];
#pragma unroll
    for (int p = 0; p < P; ++p) {
      const int r0 = (blockIdx.x * P + p) * G;
#pragma unroll
      for (int e = 0; e < 16; ++e) xs[p][e] = src[(size_t)(r0 + va) * S + e * NB + la];
    }
#pragma unroll
    for (int p = 0; p < P; ++p) {
      const int r0 = (blockIdx.x * P + p) * G;
      // ---- round A on the loaded elements
      ntt_round<LOGS, 4, MODE, false>(xs[p], 0, RB, r0 + va, k1, tw, twq, m);
      // the previous tile's LDS reads are done (at S = 256 every exchange stays inside a wave)
      if (p) tile_sync<S>();
#pragma unroll
      for (int e = 0; e < 16; ++e) lds[lidx(va, e * NB + la)] = xs[p][e];
      tile_sync<S>();
      // ---- round B
#pragma unroll
      for (int gi = 0; gi < GB; ++gi) {
        const int grp = t + gi * 256;
        const int vb = grp / 16, hb = grp % 16;
        double y[NB];
#pragma unroll
        for (int e = 0; e < NB; ++e) y[e] = lds[lidx(vb, hb * NB + e)];
        ntt_round<LOGS, RB, MODE, false>(y, hb, 0, r0 + vb, k1, tw, twq, m);
#pragma unroll
        for (int e = 0; e < NB; ++e) lds[lidx(vb, hb * NB + e)] = y[e];
      }
      tile_sync<S>();
      if (J.epi != EPI_NONE) {
        row_epilogue<G * S / 2 / 256, S>(J, l, (size_t)l * N + (size_t)r0 * S, lds, m);
      } else {
        gdbl2* d2 = (gdbl2*)(dst + (size_t)r0 * S);
#pragma unroll
        for (int q = 0; q < G * S / 2 / 256; ++q) {
          const int i = tile_pair<S>(q);
          dv2 v;
          v.x = canon(lds[lpad(2 * i)], m);
          v.y = canon(lds[lpad(2 * i + 1)], m);
          d2[i] = v;
        }
      }
    }
    }
  } else {
    // ---- round B first (low bits), loaded straight (column) or via LDS (row)
    if (MODE == NTT_ROW) {
      cgdbl2* s2 = (cgdbl2*)(src + (size_t)row0 * S);
      const bool sq = J.sq && !second;
      // every pair of the thread is requested at once (one load round trip)
      constexpr int NPP = G * S / 2 / 256;
      dv2 v[NPP];
#pragma unroll
      for (int q = 0; q < NPP; ++q) v[q] = s2[tile_pair<S>(q)];
      if (sq) {
#pragma unroll
        for (int q = 0; q < NPP; ++q) {
          v[q].x = canon(mul_mod(v[q].x, v[q].x, m), m);
          v[q].y = canon(mul_mod(v[q].y, v[q].y, m), m);
        }
      }
#pragma unroll
      for (int q = 0; q < NPP; ++q) {
        lds[lpad(2 * tile_pair<S>(q))] = v[q].x;
        lds[lpad(2 * tile_pair<S>(q) + 1)] = v[q].y;
      }
      tile_sync<S>();
      inv_row_from_lds<LOGS, G>(lds, dst, row0, k1, tw, twq, m);
      return;
    }
    if constexpr (P == 1) {
#pragma unroll
    for (int gi = 0; gi < GB; ++gi) {
      const int grp = t + gi * 256;
      const int vb = MODE == NTT_COL ? (grp % G) : (grp / 16);
      const int hb = MODE == NTT_COL ? (grp / G) : (grp % 16);
      double y[NB];
#pragma unroll
      for (int e = 0; e < NB; ++e)
        y[e] = MODE == NTT_COL ? src[gaddr(vb, hb * NB + e)] : lds[lidx(vb, hb * NB + e)];
      ntt_round<LOGS, RB, MODE, true>(y, hb, 0, row0 + vb, k1, tw, twq, m);
      // each group is read and written back by its own thread: no barrier needed here
#pragma unroll
      for (int e = 0; e < NB; ++e) lds[lidx(vb, hb * NB + e)] = y[e];
    }
    __syncthreads();
    // ---- round A, stored straight to global memory
#pragma unroll
    for (int e = 0; e < 16; ++e) x[e] = lds[lidx(va, e * NB + la)];
    ntt_round<LOGS, 4, MODE, true>(x, 0, RB, row0 + va, k1, tw, twq, m);
    // J.ek set: the last pass multiplies by ek[l] (which includes N^-1) instead of N^-1
    const double ys = (scale && J.ek) ? KPTR(J.ek)[l] : 0.0;
#pragma unroll
    for (int e = 0; e < 16; ++e) {
      double v = x[e];
      if (scale) v = J.ek ? mul_mod(red(v, m), ys, m) : mul_w(red(v, m), ni, niq, m.p);
      dst[gaddr(va, e * NB + la)] = canon_out(v, m, J.centre);
    }
    } else {
    // (the inverse column pass: every tile's loads are issued first)
    double ys[P][GB][NB];
#pragma unroll
    for (int p = 0; p < P; ++p) {
      const int cp = (blockIdx.x * P + p) * G;
#pragma unroll
      for (int gi = 0; gi < GB; ++gi) {
        const int grp = t + gi * 256;
        const int vb = grp % G, hb = grp / G;
#pragma unroll
        for (int e = 0; e < NB; ++e) ys[p][gi][e] = src[(size_t)(hb * NB + e) * C + cp + vb];
      }
    }
    // J.ek set: the last pass multiplies by ek[l] (which includes N^-1) instead of N^-1
    const double yk = (scale && J.ek) ? KPTR(J.ek)[l] : 0.0;
#pragma unroll
    for (int p = 0; p < P; ++p) {
      const int cp = (blockIdx.x * P + p) * G;
      if (p) __syncthreads();   // the previous tile's LDS reads are done
#pragma unroll
      for (int gi = 0; gi < GB; ++gi) {
        const int grp = t + gi * 256;
        const int vb = grp % G, hb = grp / G;
        ntt_round<LOGS, RB, MODE, true>(ys[p][gi], hb, 0, row0 + vb, k1, tw, twq, m);
        // each group is read and written back by its own thread: no barrier needed here
#pragma unroll
        for (int e = 0; e < NB; ++e) lds[lidx(vb, hb * NB + e)] = ys[p][gi][e];
      }
      __syncthreads();
      // ---- round A, stored straight to global memory
#pragma unroll
      for (int e = 0; e < 16; ++e) x[e] = lds[lidx(va, e * NB + la)];
      ntt_round<LOGS, 4, MODE, true>(x, 0, RB, row0 + va, k1, tw, twq, m);
#pragma unroll
      for (int e = 0; e < 16; ++e) {
        double v = x[e];
        if (scale) v = J.ek ? mul_mod(red(v, m), yk, m) : mul_w(red(v, m), ni, niq, m.p);
        dst[(size_t)(e * NB + la) * C + cp + va] = canon_out(v, m, J.centre);
      }
    }
    }
  }
}

// Row pass of the forward transform on one G x S tile (rows row0 .. row0+G-1
// of the limb at src, already through the column pass): rounds A and B as in
// k_ntt2; the transformed tile is left in LDS (lazily reduced, |v| < 2.2p).
template <int LOGS, int G>
__device__ __forceinline__ void fwd_row_tile(double* lds, cgdbl* src, int row0, int k1, kdbl* tw, kdbl* twq,
                                             const Mod& m) {
  constexpr int S = 1 << LOGS;
  constexpr int RB = LOGS - 4;
  constexpr int NB = 1 << RB;
  constexpr int GB = 16 / NB;
  const int t = threadIdx.x;
  const int va = t / NB, la = t % NB;
  double x[16];
#pragma unroll
  for (int e = 0; e < 16; ++e) x[e] = src[(size_t)(row0 + va) * S + e * NB + la];
  ntt_round<LOGS, 4, NTT_ROW, false>(x, 0, RB, row0 + va, k1, tw, twq, m);
#pragma unroll
  for (int e = 0; e < 16; ++e) lds[lpad(va * S + e * NB + la)] = x[e];
  tile_sync<S>();
#pragma unroll
  for (int gi = 0; gi < GB; ++gi) {
    const int grp = t + gi * 256;
    const int vb = grp / 16, hb = grp % 16;
    double y[NB];
#pragma unroll
    for (int e = 0; e < NB; ++e) y[e] = lds[lpad(vb * S + hb * NB + e)];
    ntt_round<LOGS, RB, NTT_ROW, false>(y, hb, 0, row0 + vb, k1, tw, twq, m);
#pragma unroll
    for (int e = 0; e < NB; ++e) lds[lpad(vb * S + hb * NB + e)] = y[e];
  }
  tile_sync<S>();
}

// Key-switch inner product fused with the row pass of the ModUp outputs'
// forward transform (N > 2^12): for extended-basis limb t and one row tile,
//   acc_w[t] = sum_j x_j[t] key_j[w][t],
// x_j[t] = d[t] (NTT domain) inside digit j, else the row pass of ext_j[t]
// (which has been through the column pass) computed here in LDS, so the
// transformed ModUp outputs never go to HBM.  Grid (row tile, job, limb).
template <int LOGS, int G>
__global__ __launch_bounds__(256) void k_inner_row(const InnerJob* __restrict__ jobs, DevTables T) {
  extern __shared__ double lds[];
  constexpr int S = 1 << LOGS;
  constexpr int NP = G * S / 2 / 256;   // pairs per thread
  const InnerJob J = jobs[blockIdx.y];
  const int t = blockIdx.z;
  if (t >= J.n_ext) return;
  const int log_n = T.log_n;
  const int N = 1 << log_n;
  const int n_mod = T.n_q + T.n_p;
  const int pr = t < J.n_chain ? t : T.n_q + (t - J.n_chain);
  const Mod m{KPTR(T.mod)[pr], KPTR(T.minv)[pr]};
  kdbl* tw = KPTR(T.psi) + (size_t)pr * N;
  kdbl* twq = KPTR(T.psiq) + (size_t)pr * N;
  const int own = t < J.n_chain ? t / J.alpha : -1;
  const int row0 = blockIdx.x * G;
  const size_t tile = (size_t)row0 * S;
  const int k1 = log_n - LOGS;
  double a0x[NP], a0y[NP], a1x[NP], a1y[NP];
#pragma unroll
  for (int q = 0; q < NP; ++q) a0x[q] = a0y[q] = a1x[q] = a1y[q] = 0.0;
  // the key tile of a digit is requested in two halves of NP/2 pairs, each
  // half at once (two round trips per digit, not one per pair), after the
  // row pass so that the loads hold no registers through the transform
  constexpr int NH = NP / 2;
  for (int j = 0; j < J.n_digits; ++j) {
    cgdbl* kb = CGPTR(J.key) + (((size_t)j * 2 + 0) * n_mod + pr) * N + tile;
    cgdbl* ka = CGPTR(J.key) + (((size_t)j * 2 + 1) * n_mod + pr) * N + tile;
    if (j != own) fwd_row_tile<LOGS, G>(lds, CGPTR(J.ext) + ((size_t)j * J.n_ext + t) * N, row0, k1, tw, twq, m);
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      dv2 kbv[NH], kav[NH], xv[NH];
#pragma unroll
      for (int r = 0; r < NH; ++r) {
        const int i = tile_pair<S>(h * NH + r);
        kbv[r] = *(cgdbl2*)(kb + 2 * i);
        kav[r] = *(cgdbl2*)(ka + 2 * i);
      }
      if (j != own) {
#pragma unroll
        for (int r = 0; r < NH; ++r) {
          const int i = tile_pair<S>(h * NH + r);
          xv[r].x = canon(lds[lpad(2 * i)], m);
          xv[r].y = canon(lds[lpad(2 * i + 1)], m);
        }
      } else {
#pragma unroll
        for (int r = 0; r < NH; ++r) {
          const double2 v = ld2(J.d, (size_t)t * N + tile + 2 * (tile_pair<S>(h * NH + r)));
          xv[r].x = v.x;
          xv[r].y = v.y;
        }
        if (J.d_square) {
#pragma unroll
          for (int r = 0; r < NH; ++r) {
            xv[r].x = canon(mul_mod(xv[r].x, xv[r].x, m), m);
            xv[r].y = canon(mul_mod(xv[r].y, xv[r].y, m), m);
          }
        }
      }
#pragma unroll
      for (int r = 0; r < NH; ++r) {
        const int q = h * NH + r;
        a0x[q] += mul_mod(xv[r].x, kbv[r].x, m);
        a0y[q] += mul_mod(xv[r].y, kbv[r].y, m);
        a1x[q] += mul_mod(xv[r].x, kav[r].x, m);
        a1y[q] += mul_mod(xv[r].y, kav[r].y, m);
        if (j & 1) {
          a0x[q] = red(a0x[q], m); a0y[q] = red(a0y[q], m);
          a1x[q] = red(a1x[q], m); a1y[q] = red(a1y[q], m);
        }
      }
    }
    // the next digit's row pass overwrites the tile in LDS
    if (j != own) tile_sync<S>();
  }
  const bool top = J.top0 && t == J.n_chain - 1;
  const double pm = top ? KPTR(J.pmq)[t] : 0.0;
#pragma unroll
  for (int q = 0; q < NP; ++q) {
    if (top) {
      const size_t o = (size_t)t * N + tile + 2 * (tile_pair<S>(q));
      double2 u0 = ld2(J.top0, o), u1 = ld2(J.top1, o);
      if (J.d_square) {
        // top0, top1 = a0, a1 of the square: d0 = a0^2, d1 = 2 a0 a1
        const double2 a0 = u0;
        u0.x = canon(mul_mod(a0.x, a0.x, m), m);
        u0.y = canon(mul_mod(a0.y, a0.y, m), m);
        u1.x = canon(mul_mod(2.0 * a0.x, u1.x, m), m);
        u1.y = canon(mul_mod(2.0 * a0.y, u1.y, m), m);
      }
      a0x[q] = red(a0x[q], m) + mul_mod(u0.x, pm, m);
      a0y[q] = red(a0y[q], m) + mul_mod(u0.y, pm, m);
      a1x[q] = red(a1x[q], m) + mul_mod(u1.x, pm, m);
      a1y[q] = red(a1y[q], m) + mul_mod(u1.y, pm, m);
    }
  }
  if (t >= J.inv_from) {
    // limbs the base conversion reads: the first pass of their inverse
    // transform runs here, on the tile in LDS
    kdbl* itw = KPTR(T.ipsi) + (size_t)pr * N;
    kdbl* itwq = KPTR(T.ipsiq) + (size_t)pr * N;
    for (int w = 0; w < 2; ++w) {
#pragma unroll
      for (int q = 0; q < NP; ++q) {
        const int i = tile_pair<S>(q);
        lds[lpad(2 * i)] = canon(w ? a1x[q] : a0x[q], m);
        lds[lpad(2 * i + 1)] = canon(w ? a1y[q] : a0y[q], m);
      }
      tile_sync<S>();
      inv_row_from_lds<LOGS, G>(lds, GPTR(J.acc) + ((size_t)w * J.n_ext + t) * N, row0, k1, itw, itwq, m);
      tile_sync<S>();
    }
    return;
  }
#pragma unroll
  for (int q = 0; q < NP; ++q) {
    const size_t o = (size_t)t * N + tile + 2 * (tile_pair<S>(q));
    st2(J.acc, o, canon(a0x[q], m), canon(a0y[q], m));
    st2(J.acc, (size_t)J.n_ext * N + o, canon(a1x[q], m), canon(a1y[q], m));
  }
}
template __global__ void k_inner_row<8, 16>(const InnerJob* __restrict__, DevTables);
template __global__ void k_inner_row<7, 32>(const InnerJob* __restrict__, DevTables);

// ModUp of one digit fused with the column pass of the forward transform of
// its outputs (N > 2^12).  src holds y_i = [x_i (D/q_i)^-1]_{q_i} for the
// digit's limbs (coefficient domain; the inverse transform of x wrote them
// scaled).  A workgroup owns one column tile and a group of EG
// extended-basis limbs e outside the digit: it streams the digit's limbs
// through registers once, accumulating
//   out_e = sum_i y_i (D/q_i) mod p_e
// for the whole group, then runs the column pass on each out_e; the result
// (ready for the row pass, which the inner product does) goes to dst limb e.
// Grid (tile, group, job): with a multiple of 8 tiles, every group of a tile
// runs on the same XCD and rereads the digit's tile from its L2.
// (one or two output limbs per workgroup fit 3 waves per SIMD without
// spilling; the compiler's default aims at 2)
template <int LOGS, int G, int EG>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(EG <= 2 ? 3 : 1, 8))) void k_modup_col(const ModUpJob* __restrict__ jobs, DevTables T) {
  extern __shared__ double lds[];
  constexpr int RB = LOGS - 4;
  constexpr int NB = 1 << RB;
  const ModUpJob J = jobs[blockIdx.z];
  const int dsz = J.digit_hi - J.digit_lo;
  const int n_out = J.n_ext - dsz;
  const int g0 = blockIdx.y * EG;
  if (g0 >= n_out) return;
  const int ng = min(EG, n_out - g0);
  const int log_n = T.log_n;
  const int N = 1 << log_n;
  const int k1 = log_n - LOGS;
  const int C = N >> LOGS;
  const int t = threadIdx.x;
  const int va = t % G, la = t / G;
  const int c0 = blockIdx.x * G;
  int ee[EG], pe[EG];
  Mod me[EG];
#pragma unroll
  for (int g = 0; g < EG; ++g) {
    const int idx = min(g0 + g, n_out - 1);
    const int e = idx < J.digit_lo ? idx : idx + dsz;   // skip the digit's own limbs
    ee[g] = e;
    pe[g] = e < J.n_chain ? e : T.n_q + (e - J.n_chain);
    me[g] = Mod{KPTR(T.mod)[pe[g]], KPTR(T.minv)[pe[g]]};
  }
  double acc[EG][16];
#pragma unroll
  for (int g = 0; g < EG; ++g)
#pragma unroll
    for (int k = 0; k < 16; ++k) acc[g][k] = 0.0;
  cgdbl* ysrc = CGPTR(J.src) + (size_t)J.digit_lo * N;
  for (int i = 0; i < dsz; ++i) {
    double y[16];
#pragma unroll
    for (int k = 0; k < 16; ++k) y[k] = ysrc[(size_t)i * N + (size_t)(k * NB + la) * C + c0 + va];
#pragma unroll
    for (int g = 0; g < EG; ++g) {
      const double c = KPTR(J.chat)[(size_t)pe[g] * dsz + i];
#pragma unroll
      for (int k = 0; k < 16; ++k) {
        acc[g][k] += mul_mod(y[k], c, me[g]);
        if (i & 1) acc[g][k] = red(acc[g][k], me[g]);
      }
    }
  }
#pragma unroll
  for (int g = 0; g < EG; ++g) {
    if (g >= ng) break;
    kdbl* tw = KPTR(T.psi) + (size_t)pe[g] * N;
    kdbl* twq = KPTR(T.psiq) + (size_t)pe[g] * N;
    double x[16];
#pragma unroll
    for (int k = 0; k < 16; ++k) x[k] = red(acc[g][k], me[g]);
    fwd_col_from_regs<LOGS, G>(x, lds, GPTR(J.dst) + (size_t)ee[g] * N, c0, k1, tw, twq, me[g]);
    // the next limb's column pass reuses the LDS tile
    __syncthreads();
  }
}
// The centred conversion B -> Q_l of the ModDown fused with the column pass
// of the forward transform of its outputs (N > 2^12): src holds
// y_b = [x_b (B/b)^-1]_b centred in (-b/2, b/2] (the inverse transform's last
// pass applied (B/b)^-1 and centred its output); a workgroup owns one column
// tile and a group of EG chain limbs t, streams the |B| source limbs through
// registers once, accumulating out_t = sum_b y_b (B/b) mod q_t for the group,
// and runs the column pass on each out_t into dst limb t.  The forward
// transform's row pass follows with the ModDown or merged combine as its
// epilogue.  Grid (tile, group, job) as for the ModUp: the groups of a tile
// share an XCD's L2.
template <int LOGS, int G, int EG>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(EG <= 2 ? 3 : 1, 8))) void k_moddown_col(const ModDownJob* __restrict__ jobs, DevTables T) {
  extern __shared__ double lds[];
  constexpr int RB = LOGS - 4;
  constexpr int NB = 1 << RB;
  const ModDownJob J = jobs[blockIdx.z];
  const int g0 = blockIdx.y * EG;
  if (g0 >= J.n_chain) return;
  const int ng = min(EG, J.n_chain - g0);
  const int extra = J.first_prime >= 0 ? 1 : 0;
  const int nb = T.n_p + extra;
  const int log_n = T.log_n;
  const int N = 1 << log_n;
  const int k1 = log_n - LOGS;
  const int C = N >> LOGS;
  const int t = threadIdx.x;
  const int va = t % G, la = t / G;
  const int c0 = blockIdx.x * G;
  int ee[EG];
  Mod me[EG];
#pragma unroll
  for (int g = 0; g < EG; ++g) {
    ee[g] = min(g0 + g, J.n_chain - 1);
    me[g] = Mod{KPTR(T.mod)[ee[g]], KPTR(T.minv)[ee[g]]};
  }
  double acc[EG][16];
#pragma unroll
  for (int g = 0; g < EG; ++g)
#pragma unroll
    for (int k = 0; k < 16; ++k) acc[g][k] = 0.0;
  for (int i = 0; i < nb; ++i) {
    double y[16];
#pragma unroll
    for (int k = 0; k < 16; ++k) y[k] = CGPTR(J.src)[(size_t)i * N + (size_t)(k * NB + la) * C + c0 + va];
#pragma unroll
    for (int g = 0; g < EG; ++g) {
      const double c = KPTR(J.chat)[(size_t)ee[g] * nb + i];
#pragma unroll
      for (int k = 0; k < 16; ++k) {
        acc[g][k] += mul_mod(y[k], c, me[g]);
        if (i & 1) acc[g][k] = red(acc[g][k], me[g]);
      }
    }
  }
#pragma unroll
  for (int g = 0; g < EG; ++g) {
    if (g >= ng) break;
    kdbl* tw = KPTR(T.psi) + (size_t)ee[g] * N;
    kdbl* twq = KPTR(T.psiq) + (size_t)ee[g] * N;
    double x[16];
#pragma unroll
    for (int k = 0; k < 16; ++k) x[k] = red(acc[g][k], me[g]);
    fwd_col_from_regs<LOGS, G>(x, lds, GPTR(J.dst) + (size_t)ee[g] * N, c0, k1, tw, twq, me[g]);
    // the next limb's column pass reuses the LDS tile
    __syncthreads();
  }
}
#define MODDOWN_INST(EG)                                                                   \
  template __global__ void k_moddown_col<8, 16, EG>(const ModDownJob* __restrict__, DevTables); \
  template __global__ void k_moddown_col<7, 32, EG>(const ModDownJob* __restrict__, DevTables); \
  template __global__ void k_moddown_col<6, 64, EG>(const ModDownJob* __restrict__, DevTables);
MODDOWN_INST(1)
MODDOWN_INST(2)
MODDOWN_INST(4)

#define MODUP_INST(EG)                                                              \
  template __global__ void k_modup_col<8, 16, EG>(const ModUpJob* __restrict__, DevTables); \
  template __global__ void k_modup_col<7, 32, EG>(const ModUpJob* __restrict__, DevTables); \
  template __global__ void k_modup_col<6, 64, EG>(const ModUpJob* __restrict__, DevTables);
MODUP_INST(1)
MODUP_INST(2)
MODUP_INST(4)

size_t ntt_lds_bytes(int logs, int g) {
  const int n = g << logs;
  return (size_t)(n + (n >> 4)) * sizeof(double);
}

#define NTT_INST(LOGS, G, MODE)                                                                  \
  template __global__ void k_ntt<LOGS, G, MODE, false>(const NttJob* __restrict__, DevTables, int); \
  template __global__ void k_ntt<LOGS, G, MODE, true>(const NttJob* __restrict__, DevTables, int);

// single pass (N <= 2^12) and two-pass halves for N = 2^13 .. 2^16
NTT_INST(10, 1, NTT_SINGLE)
NTT_INST(11, 1, NTT_SINGLE)
NTT_INST(12, 1, NTT_SINGLE)
#define NTT2_INST(LOGS, G, MODE, P)                                                                  \
  template __global__ void k_ntt2<LOGS, G, MODE, false, P>(const NttJob* __restrict__, DevTables, int); \
  template __global__ void k_ntt2<LOGS, G, MODE, true, P>(const NttJob* __restrict__, DevTables, int);
NTT2_INST(6, 64, NTT_COL, 1)
NTT2_INST(7, 32, NTT_COL, 1)
NTT2_INST(8, 16, NTT_COL, 1)
NTT2_INST(8, 16, NTT_COL, 2)
NTT2_INST(7, 32, NTT_ROW, 1)
NTT2_INST(8, 16, NTT_ROW, 1)
NTT2_INST(8, 16, NTT_ROW, 2)

void* ntt_kernel(int logs, int mode, bool inv, int* g_out, int col_tiles) {
#define PICK(LOGS, G, MODE)                                                                       \
  if (logs == LOGS && mode == MODE) {                                                             \
    *g_out = G;                                                                                   \
    return inv ? (void*)&k_ntt<LOGS, G, MODE, true> : (void*)&k_ntt<LOGS, G, MODE, false>;        \
  }
  PICK(10, 1, NTT_SINGLE)
  PICK(11, 1, NTT_SINGLE)
  PICK(12, 1, NTT_SINGLE)
#undef PICK
#define PICK2(LOGS, G, MODE, P)                                                                   \
  if (logs == LOGS && mode == MODE && col_tiles == P) {                                           \
    *g_out = G;                                                                                   \
    return inv ? (void*)&k_ntt2<LOGS, G, MODE, true, P> : (void*)&k_ntt2<LOGS, G, MODE, false, P>; \
  }
  PICK2(8, 16, NTT_COL, 2)
  PICK2(8, 16, NTT_ROW, 2)
  if (col_tiles != 1) col_tiles = 1;   // sizes without a multi-tile variant
  PICK2(6, 64, NTT_COL, 1)
  PICK2(7, 32, NTT_COL, 1)
  PICK2(8, 16, NTT_COL, 1)
  PICK2(7, 32, NTT_ROW, 1)
  PICK2(8, 16, NTT_ROW, 1)
#undef PICK2
  return nullptr;
}

// ---------------------------------------------------------------------------
// elementwise operations on limbs (NTT domain unless stated)
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(256) void k_ew(const EwJob* __restrict__ jobs, DevTables T) {
  const EwJob J = jobs[blockIdx.z];
  const int l = blockIdx.y;
  if (l >= J.n_limbs || l < J.l_first) return;
  const int pr = l < J.n_chain ? l : T.n_q + (l - J.n_chain);
  const Mod m{KPTR(T.mod)[pr], KPTR(T.minv)[pr]};
  const int N = 1 << T.log_n;
  const size_t off = (size_t)l * N;
  const double kk = J.k ? KPTR(J.k)[l] : 0.0;
  for (int i = 2 * (blockIdx.x * blockDim.x + threadIdx.x); i < N; i += 2 * gridDim.x * blockDim.x) {
    const size_t o = off + i;
    switch (J.op) {
      case EW_ADD: {
        const double2 a0 = ld2(J.a0, o), b0 = ld2(J.b0, o), a1 = ld2(J.a1, o), b1 = ld2(J.b1, o);
        st2(J.o0, o, add_mod(a0.x, b0.x, m), add_mod(a0.y, b0.y, m));
        st2(J.o1, o, add_mod(a1.x, b1.x, m), add_mod(a1.y, b1.y, m));
        break;
      }
      case EW_ADDSUB: {
        const double2 a0 = ld2(J.a0, o), b0 = ld2(J.b0, o);
        st2(J.o0, o, sub_mod(a0.x, b0.x, m), sub_mod(a0.y, b0.y, m));
        st2(J.o1, o, add_mod(a0.x, b0.x, m), add_mod(a0.y, b0.y, m));
        break;
      }
      case EW_SUB: {
        const double2 a0 = ld2(J.a0, o), b0 = ld2(J.b0, o), a1 = ld2(J.a1, o), b1 = ld2(J.b1, o);
        st2(J.o0, o, sub_mod(a0.x, b0.x, m), sub_mod(a0.y, b0.y, m));
        st2(J.o1, o, sub_mod(a1.x, b1.x, m), sub_mod(a1.y, b1.y, m));
        break;
      }
      case EW_TENSOR: {
        const double2 a0 = ld2(J.a0, o), a1 = ld2(J.a1, o), b0 = ld2(J.b0, o), b1 = ld2(J.b1, o);
        st2(J.o0, o, canon(mul_mod(a0.x, b0.x, m), m), canon(mul_mod(a0.y, b0.y, m), m));
        st2(J.o1, o, canon(mul_mod(a0.x, b1.x, m) + mul_mod(a1.x, b0.x, m), m),
            canon(mul_mod(a0.y, b1.y, m) + mul_mod(a1.y, b0.y, m), m));
        st2(J.o2, o, canon(mul_mod(a1.x, b1.x, m), m), canon(mul_mod(a1.y, b1.y, m), m));
        break;
      }
      case EW_ADD_CONST: {
        // optional operands are requested with the others (one load round trip)
        const bool cp = J.o1 != J.a1;
        const double2 a0 = ld2(J.a0, o);
        const double2 a1 = cp ? ld2(J.a1, o) : make_double2(0.0, 0.0);
        st2(J.o0, o, add_mod(a0.x, kk, m), add_mod(a0.y, kk, m));
        if (cp) st2(J.o1, o, a1.x, a1.y);
        break;
      }
      case EW_PMUL: {
        const double2 p = ld2(J.b0, o), a0 = ld2(J.a0, o), a1 = ld2(J.a1, o);
        st2(J.o0, o, canon(mul_mod(a0.x, p.x, m), m), canon(mul_mod(a0.y, p.y, m), m));
        st2(J.o1, o, canon(mul_mod(a1.x, p.x, m), m), canon(mul_mod(a1.y, p.y, m), m));
        break;
      }
      case EW_DEC2: {
        const double2 a0 = ld2(J.a0, o), a1 = ld2(J.a1, o), b0 = ld2(J.b0, o);
        st2(J.o0, o, canon(a0.x + mul_mod(a1.x, b0.x, m), m), canon(a0.y + mul_mod(a1.y, b0.y, m), m));
        break;
      }
      case EW_ENC: {
        const double2 a0 = ld2(J.a0, o), a1 = ld2(J.a1, o), b0 = ld2(J.b0, o), b1 = ld2(J.b1, o);
        st2(J.o0, o, canon(a0.x + a1.x - mul_mod(b0.x, b1.x, m), m), canon(a0.y + a1.y - mul_mod(b0.y, b1.y, m), m));
        break;
      }
      case EW_KEYB: {
        const double2 a1 = ld2(J.a1, o), b0 = ld2(J.b0, o), b1 = ld2(J.b1, o);
        const double2 c0 = kk != 0.0 ? ld2(J.c0, o) : make_double2(0.0, 0.0);
        double vx = a1.x - mul_mod(b0.x, b1.x, m), vy = a1.y - mul_mod(b0.y, b1.y, m);
        if (kk != 0.0) {
          vx += mul_mod(kk, c0.x, m);
          vy += mul_mod(kk, c0.y, m);
        }
        st2(J.o0, o, canon(vx, m), canon(vy, m));
        break;
      }
      case EW_MUL: {
        const double2 a0 = ld2(J.a0, o), b0 = ld2(J.b0, o);
        st2(J.o0, o, canon(mul_mod(a0.x, b0.x, m), m), canon(mul_mod(a0.y, b0.y, m), m));
        break;
      }
      case EW_COPY: {
        const double2 a0 = ld2(J.a0, o);
        const double2 a1 = J.o1 ? ld2(J.a1, o) : make_double2(0.0, 0.0);
        st2(J.o0, o, a0.x, a0.y);
        if (J.o1) st2(J.o1, o, a1.x, a1.y);
        break;
      }
      case EW_TENSOR2: {
        const double2 a0 = ld2(J.a0, o), a1 = ld2(J.a1, o), b0 = ld2(J.b0, o), b1 = ld2(J.b1, o);
        const double2 z2 = make_double2(0.0, 0.0);
        const double2 c0 = J.c0 ? ld2(J.c0, o) : z2, c1 = J.c0 ? ld2(J.c1, o) : z2;
        const double2 e0 = J.c0 ? ld2(J.e0, o) : z2, e1 = J.c0 ? ld2(J.e1, o) : z2;
        const double2 f0 = J.f0 ? ld2(J.f0, o) : z2, f1 = J.f0 ? ld2(J.f1, o) : z2;
        const double2 g0 = J.g0 ? ld2(J.g0, o) : z2, g1 = J.g0 ? ld2(J.g1, o) : z2;
        double r0x = mul_mod(a0.x, b0.x, m), r0y = mul_mod(a0.y, b0.y, m);
        double r1x = mul_mod(a0.x, b1.x, m) + mul_mod(a1.x, b0.x, m);
        double r1y = mul_mod(a0.y, b1.y, m) + mul_mod(a1.y, b0.y, m);
        double r2x = mul_mod(a1.x, b1.x, m), r2y = mul_mod(a1.y, b1.y, m);
        if (J.c0) {
          r0x += mul_mod(c0.x, e0.x, m);
          r0y += mul_mod(c0.y, e0.y, m);
          r1x = red(r1x, m) + mul_mod(c0.x, e1.x, m) + mul_mod(c1.x, e0.x, m);
          r1y = red(r1y, m) + mul_mod(c0.y, e1.y, m) + mul_mod(c1.y, e0.y, m);
          r2x += mul_mod(c1.x, e1.x, m);
          r2y += mul_mod(c1.y, e1.y, m);
        }
        if (J.f0) {
          double fx0 = f0.x, fy0 = f0.y, fx1 = f1.x, fy1 = f1.y;
          if (J.k) {
            // the addend is a constant combination, formed as EW_LIN2 forms it
            fx0 = mul_mod(f0.x, kk, m); fy0 = mul_mod(f0.y, kk, m);
            fx1 = mul_mod(f1.x, kk, m); fy1 = mul_mod(f1.y, kk, m);
            if (J.g0) {
              const double k2 = KPTR(J.k2)[l];
              fx0 += mul_mod(g0.x, k2, m); fy0 += mul_mod(g0.y, k2, m);
              fx1 += mul_mod(g1.x, k2, m); fy1 += mul_mod(g1.y, k2, m);
            }
            fx0 = canon(fx0, m); fy0 = canon(fy0, m);
            fx1 = canon(fx1, m); fy1 = canon(fy1, m);
          }
          r0x += fx0;
          r0y += fy0;
          r1x = red(r1x, m) + fx1;
          r1y = red(r1y, m) + fy1;
        }
        st2(J.o0, o, canon(r0x, m), canon(r0y, m));
        st2(J.o1, o, canon(r1x, m), canon(r1y, m));
        st2(J.o2, o, canon(r2x, m), canon(r2y, m));
        break;
      }
      case EW_PADD: {
        const bool cp = J.o1 != J.a1;
        const double2 a0 = ld2(J.a0, o), p = ld2(J.b0, o);
        const double2 a1 = cp ? ld2(J.a1, o) : make_double2(0.0, 0.0);
        st2(J.o0, o, add_mod(a0.x, p.x, m), add_mod(a0.y, p.y, m));
        if (cp) st2(J.o1, o, a1.x, a1.y);
        break;
      }
      case EW_PMAC: {
        const double2 p = ld2(J.b0, o), a0 = ld2(J.a0, o), a1 = ld2(J.a1, o), c0 = ld2(J.c0, o), c1 = ld2(J.c1, o);
        st2(J.o0, o, canon(mul_mod(a0.x, p.x, m) + c0.x, m), canon(mul_mod(a0.y, p.y, m) + c0.y, m));
        st2(J.o1, o, canon(mul_mod(a1.x, p.x, m) + c1.x, m), canon(mul_mod(a1.y, p.y, m) + c1.y, m));
        break;
      }
      case EW_LIN2: {
        const double2 a0 = ld2(J.a0, o), a1 = ld2(J.a1, o);
        const double2 b0 = J.b0 ? ld2(J.b0, o) : make_double2(0.0, 0.0);
        const double2 b1 = J.b0 ? ld2(J.b1, o) : make_double2(0.0, 0.0);
        double r0x = mul_mod(a0.x, kk, m), r0y = mul_mod(a0.y, kk, m);
        double r1x = mul_mod(a1.x, kk, m), r1y = mul_mod(a1.y, kk, m);
        if (J.b0) {
          const double k2 = KPTR(J.k2)[l];
          r0x += mul_mod(b0.x, k2, m);
          r0y += mul_mod(b0.y, k2, m);
          r1x += mul_mod(b1.x, k2, m);
          r1y += mul_mod(b1.y, k2, m);
        }
        st2(J.o0, o, canon(r0x, m), canon(r0y, m));
        st2(J.o1, o, canon(r1x, m), canon(r1y, m));
        break;
      }
      default:
        break;
    }
  }
}

// ---------------------------------------------------------------------------
// basis conversion (hybrid key switching)
// ModUp for one digit D = prod_{i in digit} q_i:
//   y_i = [x_i (D/q_i)^-1]_{q_i},  out_t = sum_i y_i (D/q_i) mod t
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(256) void k_modup(const ModUpJob* __restrict__ jobs, DevTables T) {
  const ModUpJob J = jobs[blockIdx.z];
  const int N = 1 << T.log_n;
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= N) return;
  const int dsz = J.digit_hi - J.digit_lo;
  double y[MAX_DIGIT];
#pragma unroll
  for (int i = 0; i < MAX_DIGIT; ++i) {
    if (i < dsz) {
      const int pr = J.digit_lo + i;
      const Mod mi{KPTR(T.mod)[pr], KPTR(T.minv)[pr]};
      y[i] = canon(mul_mod(CGPTR(J.src)[(size_t)pr * N + k], KPTR(J.cinv)[i], mi), mi);
    }
  }
  for (int t = 0; t < J.n_ext; ++t) {
    if (t >= J.digit_lo && t < J.digit_hi) continue;
    const int pr = t < J.n_chain ? t : T.n_q + (t - J.n_chain);
    const Mod mt{KPTR(T.mod)[pr], KPTR(T.minv)[pr]};
    kdbl* ch = KPTR(J.chat) + (size_t)pr * dsz;
    double acc = 0.0;
#pragma unroll
    for (int i = 0; i < MAX_DIGIT; ++i) {
      if (i < dsz) {
        acc += mul_mod(y[i], ch[i], mt);
        if (i & 1) acc = red(acc, mt);
      }
    }
    GPTR(J.dst)[(size_t)t * N + k] = canon(acc, mt);
  }
}

// Conv_{P -> Q_l}: y_k = [x_k (P/p_k)^-1]_{p_k},  out_i = sum_k y_k (P/p_k) mod q_i
__global__ __launch_bounds__(256) void k_moddown_conv(const ModDownJob* __restrict__ jobs, DevTables T) {
  const ModDownJob J = jobs[blockIdx.z];
  const int N = 1 << T.log_n;
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= N) return;
  const int extra = J.first_prime >= 0 ? 1 : 0;
  const int nb = T.n_p + extra;
  // digits [x_b (B/b)^-1]_b taken centred, in (-b/2, b/2), so the conversion
  // overshoots by a signed multiple of B and the division rounds without bias
  // all source limbs are requested before any is used (one load round trip)
  double y[MAX_DIGIT + 1];
#pragma unroll
  for (int i = 0; i < MAX_DIGIT + 1; ++i)
    if (i < nb) y[i] = CGPTR(J.src)[(size_t)i * N + k];
#pragma unroll
  for (int i = 0; i < MAX_DIGIT + 1; ++i) {
    if (i < nb) {
      const int pr = i < extra ? J.first_prime : T.n_q + i - extra;
      const Mod mi{KPTR(T.mod)[pr], KPTR(T.minv)[pr]};
      const double z = J.cinv ? canon(mul_mod(y[i], KPTR(J.cinv)[i], mi), mi) : y[i];
      y[i] = 2.0 * z > mi.p ? z - mi.p : z;
    }
  }
  for (int t = 0; t < J.n_chain; ++t) {
    const Mod mt{KPTR(T.mod)[t], KPTR(T.minv)[t]};
    kdbl* ch = KPTR(J.chat) + (size_t)t * nb;
    double acc = 0.0;
#pragma unroll
    for (int i = 0; i < MAX_DIGIT + 1; ++i) {
      if (i < nb) {
        acc += mul_mod(y[i], ch[i], mt);
        if (i & 1) acc = red(acc, mt);
      }
    }
    GPTR(J.dst)[(size_t)t * N + k] = canon(acc, mt);
  }
}

// acc_w[t] = sum_j x_j[t] key_j[w][t]; x_j[t] = d[t] inside digit j, else ModUp output.
// Grid (tile, job, limb): with a multiple of 8 tiles per limb, one tile of a
// key limb lands on the same XCD for every job of the batch (relinearisation
// shares one key across the batch), so its L2 serves the repeats.
__global__ __launch_bounds__(256) void k_inner(const InnerJob* __restrict__ jobs, DevTables T) {
  const InnerJob J = jobs[blockIdx.y];
  const int t = blockIdx.z;
  if (t >= J.n_ext) return;
  const int N = 1 << T.log_n;
  const int n_mod = T.n_q + T.n_p;
  const int pr = t < J.n_chain ? t : T.n_q + (t - J.n_chain);
  const Mod m{KPTR(T.mod)[pr], KPTR(T.minv)[pr]};
  const int own = t < J.n_chain ? t / J.alpha : -1;
  for (int k = 2 * (blockIdx.x * blockDim.x + threadIdx.x); k < N; k += 2 * gridDim.x * blockDim.x) {
    double a0x = 0.0, a0y = 0.0, a1x = 0.0, a1y = 0.0;
    for (int j = 0; j < J.n_digits; ++j) {
      const double2 x = (j == own) ? ld2(J.d, (size_t)t * N + k) : ld2(J.ext, ((size_t)j * J.n_ext + t) * N + k);
      const double2 kb = ld2(J.key, (((size_t)j * 2 + 0) * n_mod + pr) * N + k);
      const double2 ka = ld2(J.key, (((size_t)j * 2 + 1) * n_mod + pr) * N + k);
      a0x += mul_mod(x.x, kb.x, m);
      a0y += mul_mod(x.y, kb.y, m);
      a1x += mul_mod(x.x, ka.x, m);
      a1y += mul_mod(x.y, ka.y, m);
      if (j & 1) {
        a0x = red(a0x, m); a0y = red(a0y, m); a1x = red(a1x, m); a1y = red(a1y, m);
      }
    }
    if (J.top0 && t == J.n_chain - 1) {
      const double pm = KPTR(J.pmq)[t];
      const double2 u0 = ld2(J.top0, (size_t)t * N + k), u1 = ld2(J.top1, (size_t)t * N + k);
      a0x = red(a0x, m) + mul_mod(u0.x, pm, m);
      a0y = red(a0y, m) + mul_mod(u0.y, pm, m);
      a1x = red(a1x, m) + mul_mod(u1.x, pm, m);
      a1y = red(a1y, m) + mul_mod(u1.y, pm, m);
    }
    st2(J.acc, (size_t)t * N + k, canon(a0x, m), canon(a0y, m));
    st2(J.acc, ((size_t)J.n_ext + t) * N + k, canon(a1x, m), canon(a1y, m));
  }
}

// X -> X^g in the bit-reversed NTT domain: out[k] = in[brv(((2 brv(k) + 1) g mod 2N - 1) / 2)]
__global__ __launch_bounds__(256) void k_automorph(const AutoJob* __restrict__ jobs, DevTables T) {
  const AutoJob J = jobs[blockIdx.z];
  const int l = blockIdx.y;
  if (l >= J.n_limbs) return;
  const int log_n = T.log_n;
  const int N = 1 << log_n;
  const uint32_t mask = 2u * N - 1u;
  const double* src = J.src + (size_t)l * N;
  double* dst = J.dst + (size_t)l * N;
  for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < N; k += gridDim.x * blockDim.x) {
    const uint32_t kr = __builtin_bitreverse32((uint32_t)k) >> (32 - log_n);
    const uint32_t e = ((2u * kr + 1u) * J.galois) & mask;
    const uint32_t j = (e - 1u) >> 1;
    const uint32_t s = __builtin_bitreverse32(j) >> (32 - log_n);
    dst[k] = src[s];
  }
}

// CRT lift of m from residues r0 mod q0, r1 mod q1 (coefficient domain) to the
// centred integer, then m mod q_t for t < n_out; optionally the int64 value.
// ctab: [n_out][2] = (q0 mod q_t, q0 q1 mod q_t); cinv = q0^-1 mod q1.
__global__ __launch_bounds__(256) void k_lift(const LiftJob* __restrict__ jobs, DevTables T, const double* __restrict__ ctab,
                                              double q0inv_q1) {
  const LiftJob J = jobs[blockIdx.z];
  const int N = 1 << T.log_n;
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= N) return;
  const Mod m0{KPTR(T.mod)[0], KPTR(T.minv)[0]};
  const Mod m1{KPTR(T.mod)[1], KPTR(T.minv)[1]};
  const double r0 = J.r0[k], r1 = J.r1[k];
  const double diff = r1 - red(r0, m1);
  const double d = canon(mul_mod(diff, q0inv_q1, m1), m1);
  const double h = (m1.p - 1.0) * 0.5;
  const bool neg = d > h || (d == h && r0 > (m0.p - 1.0) * 0.5);
  for (int t = 0; t < J.n_out; ++t) {
    const Mod mt{KPTR(T.mod)[t], KPTR(T.minv)[t]};
    double v = red(r0, mt) + mul_mod(d, ctab[2 * t], mt);
    if (neg) v -= ctab[2 * t + 1];
    J.dst[(size_t)t * N + k] = canon(v, mt);
  }
  if (J.m_out) {
    const uint64_t q0 = (uint64_t)m0.p, q1 = (uint64_t)m1.p;
    const uint64_t di = (uint64_t)d, ri = (uint64_t)r0;
    uint64_t lo = q0 * di;
    uint64_t hi = __umul64hi(q0, di);
    const uint64_t lo2 = lo + ri;
    hi += lo2 < lo;
    lo = lo2;
    if (neg) {
      const uint64_t Qlo = q0 * q1, Qhi = __umul64hi(q0, q1);
      const uint64_t nlo = lo - Qlo;
      hi = hi - Qhi - (lo < Qlo);
      lo = nlo;
    }
    // (hi, lo) is a two's-complement 128-bit value; keep it when it fits int64
    const int64_t v = (int64_t)lo;
    const bool fits = (hi == 0 && v >= 0) || (hi == ~0ull && v < 0);
    J.m_out[k] = fits ? v : INT64_MIN;
  }
}

// Baby-step giant-step inner sums of one linear-transform group: every input
// x_b is read once, every plaintext once, every output written once (the
// per-baby-step multiply-accumulate reads and writes each output n1 times).
// Two residues per thread; partial sums are reduced after every term.
__global__ __launch_bounds__(256) void k_bsgs(const BsgsJob* __restrict__ jobs, DevTables T) {
  const BsgsJob& J = jobs[blockIdx.z];
  const int l = blockIdx.y;
  if (l >= J.n_limbs) return;
  const Mod m{KPTR(T.mod)[l], KPTR(T.minv)[l]};
  const int N = 1 << T.log_n;
  const size_t off = (size_t)l * N;
  const int n1 = J.n1, ng = J.n_giants;
  for (int i = 2 * (blockIdx.x * blockDim.x + threadIdx.x); i < N; i += 2 * gridDim.x * blockDim.x) {
    const size_t o = off + i;
    double2 xa[8], xb[8];
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      if (b < n1) {
        xa[b] = ld2(J.x0[b], o);
        xb[b] = ld2(J.x1[b], o);
      } else {
        xa[b] = make_double2(0.0, 0.0);
        xb[b] = make_double2(0.0, 0.0);
      }
    }
#pragma unroll
    for (int g = 0; g < 8; ++g) {
      if (g >= ng) break;
      double a0x = 0.0, a0y = 0.0, a1x = 0.0, a1y = 0.0;
#pragma unroll
      for (int b = 0; b < 8; ++b) {
        const double* pp = J.pt[g * 8 + b];
        if (b >= n1 || !pp) continue;
        const double2 p = ld2(pp, o);
        a0x = red(a0x + mul_mod(xa[b].x, p.x, m), m);
        a0y = red(a0y + mul_mod(xa[b].y, p.y, m), m);
        a1x = red(a1x + mul_mod(xb[b].x, p.x, m), m);
        a1y = red(a1y + mul_mod(xb[b].y, p.y, m), m);
      }
      st2(J.o0[g], o, canon(a0x, m), canon(a0y, m));
      st2(J.o1[g], o, canon(a1x, m), canon(a1y, m));
    }
  }
}

// ModRaise: residue r mod q_0 -> centred value v in (-q_0/2, q_0/2] -> v mod q_t
__global__ __launch_bounds__(256) void k_raise(const RaiseJob* __restrict__ jobs, DevTables T) {
  const RaiseJob J = jobs[blockIdx.z];
  const int N = 1 << T.log_n;
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= N) return;
  const double q0 = KPTR(T.mod)[0];
  const double r = J.src[k];
  const double v = r > (q0 - 1.0) * 0.5 ? r - q0 : r;
  for (int t = 0; t < J.n_out; ++t) {
    const Mod mt{KPTR(T.mod)[t], KPTR(T.minv)[t]};
    J.dst[(size_t)t * N + k] = canon(v, mt);
  }
}

// ---------------------------------------------------------------------------
// counter-based SplitMix64 (Steele, Lea, Flood 2014) and samplers
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint64_t sm_mix(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}
__device__ __forceinline__ uint64_t sm_draw(uint64_t key, uint64_t i) { return sm_mix(key + (i + 1) * 0x9E3779B97F4A7C15ull); }

__global__ __launch_bounds__(256) void k_sample(const SampleJob* __restrict__ jobs, DevTables T) {
  const SampleJob J = jobs[blockIdx.z];
  const int l = blockIdx.y;
  if (l >= J.n_limbs) return;
  const int pr = l < J.n_chain ? l : T.n_q + (l - J.n_chain);
  const int N = 1 << T.log_n;
  const Mod m{KPTR(T.mod)[pr], KPTR(T.minv)[pr]};
  const uint64_t tag = J.kind == SAMPLE_UNIFORM ? (J.tag_base | (uint64_t)pr) : (J.tag_base | 0xFFFull);
  const uint64_t key = sm_mix(J.seed ^ sm_mix(tag));
  const uint64_t q = (uint64_t)m.p;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < N; i += gridDim.x * blockDim.x) {
    double v;
    if (J.kind == SAMPLE_UNIFORM) {
      const uint64_t hi = sm_draw(key, 2 * (uint64_t)i), lo = sm_draw(key, 2 * (uint64_t)i + 1);
      const uint64_t a = __umul64hi(lo, q);
      const uint64_t b_lo = hi * q;
      const uint64_t b_hi = __umul64hi(hi, q);
      const uint64_t s = b_lo + a;
      v = (double)(b_hi + (s < b_lo));
    } else if (J.kind == SAMPLE_CBD) {
      const uint64_t r = sm_draw(key, (uint64_t)i);
      const uint64_t mk = (1ull << 21) - 1;
      v = (double)((int)__popcll(r & mk) - (int)__popcll((r >> 21) & mk));
      v = v < 0.0 ? v + m.p : v;
    } else if (J.kind == SAMPLE_SPARSE) {
      const uint64_t r = sm_draw(key, (uint64_t)i);
      v = (r >> (64 - T.log_n)) < (uint64_t)J.param ? ((r & 1ull) ? m.p - 1.0 : 1.0) : 0.0;
    } else {
      const uint64_t r = sm_draw(key, (uint64_t)i);
      v = (double)(int64_t)__umul64hi(r, 3ull) - 1.0;
      v = v < 0.0 ? v + m.p : v;
    }
    J.dst[(size_t)l * N + i] = v;
  }
}

// int64 polynomial -> canonical residues per limb
__global__ __launch_bounds__(256) void k_int_spread(const IntSpreadJob* __restrict__ jobs, DevTables T) {
  const IntSpreadJob J = jobs[blockIdx.z];
  const int l = blockIdx.y;
  if (l >= J.n_limbs) return;
  const int pr = l < J.n_chain ? l : T.n_q + (l - J.n_chain);
  const int N = 1 << T.log_n;
  const int64_t q = (int64_t)T.mod[pr];
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < N; i += gridDim.x * blockDim.x) {
    int64_t r = J.src[i] % q;
    if (r < 0) r += q;
    J.dst[(size_t)l * N + i] = (double)r;
  }
}

// ---------------------------------------------------------------------------
// canonical-embedding encode in double-double (Dekker 1971; Shewchuk 1997):
// m_k = round-half-away(scale * 2/N * sum_j z_j cos(pi (5^j k mod 2N) / N))
// ---------------------------------------------------------------------------
__device__ __forceinline__ void two_sum(double a, double b, double& s, double& e) {
  s = a + b;
  const double bb = s - a;
  e = (a - (s - bb)) + (b - bb);
}
__device__ __forceinline__ void dd_add(double& ah, double& al, double bh, double bl) {
  double s, e;
  two_sum(ah, bh, s, e);
  e += al + bl;
  ah = s + e;
  al = e - (ah - s);
}
__device__ __forceinline__ void dd_mul(double ah, double al, double bh, double bl, double& ph, double& pl) {
  const double p = ah * bh;
  double e = fma_rn(ah, bh, -p);
  e = fma_rn(ah, bl, e);
  e = fma_rn(al, bh, e);
  ph = p + e;
  pl = e - (ph - p);
}
// (sh + sl)(kh + kl) rounded half away from zero, as an integer
__device__ __forceinline__ int64_t dd_scale_round(double sh, double sl, double kh, double kl) {
  double yh, yl;
  dd_mul(sh, sl, kh, kl, yh, yl);
  const bool negv = yh < 0.0 || (yh == 0.0 && yl < 0.0);
  if (negv) { yh = -yh; yl = -yl; }
  const double f = floor(yh);
  const double frac = (yh - f) + yl + 0.5;
  const int64_t v = (int64_t)f + (int64_t)floor(frac);
  return negv ? -v : v;
}

__global__ __launch_bounds__(256) void k_encode(const EncodeJob* __restrict__ jobs, DevTables T) {
  const EncodeJob J = jobs[blockIdx.z];
  const int log_n = T.log_n;
  const int N = 1 << log_n;
  const uint32_t mask = 2u * N - 1u;
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= N) return;
  double sh = 0.0, sl = 0.0;
  uint32_t g = 1;
  // sin(pi t / N) = cos(pi (t + 3N/2) / N)
  const uint32_t quarter = 3u * (uint32_t)N / 2u;
  for (int j = 0; j < J.nnz; ++j) {
    const double z = J.z[j];
    const double zi = J.zi ? J.zi[j] : 0.0;
    const uint32_t gj = J.gs ? J.gs[j] : g;
    const uint32_t t = (gj * (uint32_t)k) & mask;
    if (z != 0.0) {
      double ph, pl;
      dd_mul(z, 0.0, T.cos_hi[t], T.cos_lo[t], ph, pl);
      dd_add(sh, sl, ph, pl);
    }
    if (zi != 0.0) {
      const uint32_t ts = (t + quarter) & mask;
      double ph, pl;
      dd_mul(zi, 0.0, T.cos_hi[ts], T.cos_lo[ts], ph, pl);
      dd_add(sh, sl, ph, pl);
    }
    g = (g * 5u) & mask;
  }
  J.m[k] = dd_scale_round(sh, sl, J.scale_hi, J.scale_lo);
}

// ---- dense encoding through a length-2N Stockham FFT (FftEncJob) ----
// phase -2: zero the first plane set; -1: scatter A; s >= 0: radix-2 stage s
// (butterfly j: p = j >> s, q = j mod 2^s, length-2N data, m = N >> s):
//   y[q + 2^s 2p] = a + b,  y[q + 2^s (2p+1)] = (a - b) w^(p 2^s),  w = e^(i pi / N),
//   a = x[q + 2^s p], b = x[q + 2^s (p + m)]   (ping-pong between the plane sets);
// phase 1000: Re X[k] for k < N, scaled and rounded half away from zero.
__global__ __launch_bounds__(256) void k_fft_enc(const FftEncJob* __restrict__ jobs, DevTables T, int phase) {
  const FftEncJob J = jobs[blockIdx.y];
  const int log_n = T.log_n;
  const int N = 1 << log_n;
  const int L = 2 * N;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  double* P0 = J.buf;
  double* P1 = J.buf + 4 * (size_t)L;
  if (phase == -2) {
    if (i < L) P0[i] = P0[L + i] = P0[2 * L + i] = P0[3 * L + i] = 0.0;
    return;
  }
  if (phase == -1) {
    if (i < J.nnz) {
      const uint32_t t = J.gs[i];
      P0[t] = J.z[i];
      P0[2 * L + t] = -J.zi[i];
    }
    return;
  }
  if (phase == 1000) {
    if (i >= N) return;
    const double* X = ((log_n + 1) & 1) ? P1 : P0;   // log2(2N) stages
    J.m[i] = dd_scale_round(X[i], X[L + i], J.scale_hi, J.scale_lo);
    return;
  }
  const int st = phase;
  if (i >= N) return;
  const double* x = (st & 1) ? P1 : P0;
  double* y = (st & 1) ? P0 : P1;
  const int sp = 1 << st;
  const int p = i >> st, q = i & (sp - 1);
  const int m = N >> st;
  const int ia = q + sp * p, ib = q + sp * (p + m);
  const int o0 = q + sp * 2 * p, o1 = o0 + sp;
  double arh = x[ia], arl = x[L + ia], aih = x[2 * L + ia], ail = x[3 * L + ia];
  const double brh = x[ib], brl = x[L + ib], bih = x[2 * L + ib], bil = x[3 * L + ib];
  // difference first (a is overwritten by the sum)
  double drh = arh, drl = arl, dih = aih, dil = ail;
  dd_add(drh, drl, -brh, -brl);
  dd_add(dih, dil, -bih, -bil);
  dd_add(arh, arl, brh, brl);
  dd_add(aih, ail, bih, bil);
  y[o0] = arh; y[L + o0] = arl; y[2 * L + o0] = aih; y[3 * L + o0] = ail;
  const uint32_t mask = (uint32_t)L - 1u;
  const uint32_t t = ((uint32_t)p << st) & mask;
  const uint32_t ts = (t + 3u * (uint32_t)N / 2u) & mask;
  const double wrh = T.cos_hi[t], wrl = T.cos_lo[t], wih = T.cos_hi[ts], wil = T.cos_lo[ts];
  // (dr + i di)(wr + i wi) = (dr wr - di wi) + i (dr wi + di wr)
  double rh, rl, uh, ul;
  dd_mul(drh, drl, wrh, wrl, rh, rl);
  dd_mul(dih, dil, wih, wil, uh, ul);
  dd_add(rh, rl, -uh, -ul);
  double ih, il, vh, vl;
  dd_mul(drh, drl, wih, wil, ih, il);
  dd_mul(dih, dil, wrh, wrl, vh, vl);
  dd_add(ih, il, vh, vl);
  y[o1] = rh; y[L + o1] = rl; y[2 * L + o1] = ih; y[3 * L + o1] = il;
}

// decode of slots [0, nslots): z_j = (1/scale) sum_k m_k cos(pi (5^j k mod 2N) / N)
__global__ __launch_bounds__(256) void k_decode(const int64_t* __restrict__ m, double* __restrict__ z, double inv_scale,
                                                DevTables T) {
  __shared__ double part[256];
  const int log_n = T.log_n;
  const int N = 1 << log_n;
  const uint32_t mask = 2u * N - 1u;
  const int j = blockIdx.x;
  uint32_t g = 1;
  for (int i = 0; i < j; ++i) g = (g * 5u) & mask;
  double acc = 0.0;
  for (int k = threadIdx.x; k < N; k += blockDim.x) {
    const uint32_t t = (g * (uint32_t)k) & mask;
    acc += (double)m[k] * T.cos_hi[t];
  }
  part[threadIdx.x] = acc;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) part[threadIdx.x] += part[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) z[j] = part[0] * inv_scale;
}

}  // namespace secpe

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
namespace secpe {

static inline int ew_blocks(int n) { return (n + 256 * 2 - 1) / (256 * 2); }

int ntt_pass_count(const DevTables& T) { return T.log_n <= 12 ? 1 : 2; }

// one pass of the negacyclic NTT over every job: a single pass for N <= 2^12;
// otherwise N = 2^k1 x 2^k2 with pass 0 = columns then rows (forward) or rows
// then columns (inverse); the second pass works in place on what the first
// wrote to dst
void launch_ntt_pass(const DevTables& T, bool inverse, const NttJob* jobs, int n_jobs, int max_limbs, int pass,
                     hipStream_t s, int tiles_sched) {
  if (n_jobs <= 0 || max_limbs <= 0) return;
  const int log_n = T.log_n;
  const int N = 1 << log_n;
  const int k1 = log_n / 2, k2 = log_n - k1;
  int logs, mode;
  if (log_n <= 12) {
    logs = log_n;
    mode = NTT_SINGLE;
  } else if (!inverse) {
    logs = pass == 0 ? k1 : k2;
    mode = pass == 0 ? NTT_COL : NTT_ROW;
  } else {
    logs = pass == 0 ? k2 : k1;
    mode = pass == 0 ? NTT_ROW : NTT_COL;
  }
  int g = 0;
  // two tiles per workgroup where the schedule asks for it and a variant exists
  const int bit = mode == NTT_COL ? (inverse ? 2 : 1) : (inverse ? 0 : 4);
  int p = logs == 8 && (tiles_sched & bit) ? 2 : 1;
  void* fn = ntt_kernel(logs, mode, inverse, &g, p);
  const int tiles = (N >> logs) / g / p;
  // limb-major: consecutive workgroups transform the same limb (prime) of
  // successive jobs, so that prime's twiddles are reused from L2
  dim3 grid(tiles, n_jobs, max_limbs);
  const NttJob* jp = jobs;
  DevTables t = T;
  int sec = log_n <= 12 ? 0 : pass;
  void* args[] = {(void*)&jp, (void*)&t, (void*)&sec};
  (void)hipLaunchKernel(fn, grid, dim3(256), args, ntt_lds_bytes(logs, g), s);
}

bool inner_row_fused(const DevTables& T) { return T.log_n > 12; }

// A column-fused base conversion whose grid (tile, output group, job) would
// hold fewer than two workgroups per CU at eg output limbs per workgroup takes
// one limb per workgroup instead: a single query's conversions then still fill
// the chip (the source tiles, read once per group, are few and stay in L2).
// Every eg gives the same residues.
static int conv_eg(int eg, int tiles, int max_out, int n_jobs) {
  eg = eg == 2 ? 2 : 4;
  return (long)tiles * ((max_out + eg - 1) / eg) * n_jobs < 512 ? 1 : eg;
}

void launch_modup_col(const DevTables& T, const ModUpJob* jobs, int n_jobs, int max_ext, int eg, hipStream_t s) {
  if (n_jobs <= 0 || max_ext <= 0) return;
  const int log_n = T.log_n;
  const int k1 = log_n / 2;   // column length of the two-pass split
  const int g = k1 == 8 ? 16 : k1 == 7 ? 32 : 64;
  eg = conv_eg(eg, (1 << (log_n - k1)) / g, max_ext, n_jobs);
  // max_ext bounds the output limbs of a job (n_ext minus its digit)
  dim3 grid((1 << (log_n - k1)) / g, (max_ext + eg - 1) / eg, n_jobs);
  const size_t lds = ntt_lds_bytes(k1, g);
#define LAUNCH_MODUP(EG)                                                                         \
  if (k1 == 8) hipLaunchKernelGGL((k_modup_col<8, 16, EG>), grid, dim3(256), lds, s, jobs, T);     \
  else if (k1 == 7) hipLaunchKernelGGL((k_modup_col<7, 32, EG>), grid, dim3(256), lds, s, jobs, T); \
  else hipLaunchKernelGGL((k_modup_col<6, 64, EG>), grid, dim3(256), lds, s, jobs, T);
  if (eg == 1) {
    LAUNCH_MODUP(1)
  } else if (eg == 2) {
    LAUNCH_MODUP(2)
  } else {
    LAUNCH_MODUP(4)
  }
#undef LAUNCH_MODUP
}

void launch_moddown_col(const DevTables& T, const ModDownJob* jobs, int n_jobs, int max_chain, int eg,
                        hipStream_t s) {
  if (n_jobs <= 0 || max_chain <= 0) return;
  const int log_n = T.log_n;
  const int k1 = log_n / 2;   // column length of the two-pass split
  const int g = k1 == 8 ? 16 : k1 == 7 ? 32 : 64;
  eg = conv_eg(eg, (1 << (log_n - k1)) / g, max_chain, n_jobs);
  dim3 grid((1 << (log_n - k1)) / g, (max_chain + eg - 1) / eg, n_jobs);
  const size_t lds = ntt_lds_bytes(k1, g);
#define LAUNCH_MODDOWN(EG)                                                                          \
  if (k1 == 8) hipLaunchKernelGGL((k_moddown_col<8, 16, EG>), grid, dim3(256), lds, s, jobs, T);     \
  else if (k1 == 7) hipLaunchKernelGGL((k_moddown_col<7, 32, EG>), grid, dim3(256), lds, s, jobs, T); \
  else hipLaunchKernelGGL((k_moddown_col<6, 64, EG>), grid, dim3(256), lds, s, jobs, T);
  if (eg == 1) {
    LAUNCH_MODDOWN(1)
  } else if (eg == 2) {
    LAUNCH_MODDOWN(2)
  } else {
    LAUNCH_MODDOWN(4)
  }
#undef LAUNCH_MODDOWN
}

void launch_inner_row(const DevTables& T, const InnerJob* jobs, int n_jobs, int max_ext, hipStream_t s) {
  if (n_jobs <= 0 || max_ext <= 0) return;
  const int log_n = T.log_n;
  const int k2 = log_n - log_n / 2;   // row length of the two-pass split
  const int g = k2 == 8 ? 16 : 32;
  dim3 grid((1 << (log_n - k2)) / g, n_jobs, max_ext);
  if (k2 == 8) hipLaunchKernelGGL((k_inner_row<8, 16>), grid, dim3(256), ntt_lds_bytes(8, 16), s, jobs, T);
  else hipLaunchKernelGGL((k_inner_row<7, 32>), grid, dim3(256), ntt_lds_bytes(7, 32), s, jobs, T);
}

void launch_ntt(const DevTables& T, bool inverse, const NttJob* jobs, int n_jobs, int max_limbs, hipStream_t s,
                int tiles_sched) {
  for (int p = 0; p < ntt_pass_count(T); ++p) launch_ntt_pass(T, inverse, jobs, n_jobs, max_limbs, p, s, tiles_sched);
}

void launch_ew(const DevTables& T, const EwJob* jobs, int n_jobs, int max_limbs, hipStream_t s) {
  if (n_jobs <= 0 || max_limbs <= 0) return;
  dim3 grid(ew_blocks(1 << T.log_n), max_limbs, n_jobs);
  hipLaunchKernelGGL(k_ew, grid, dim3(256), 0, s, jobs, T);
}
void launch_modup(const DevTables& T, const ModUpJob* jobs, int n_jobs, hipStream_t s) {
  if (n_jobs <= 0) return;
  dim3 grid((1 << T.log_n) / 256, 1, n_jobs);
  hipLaunchKernelGGL(k_modup, grid, dim3(256), 0, s, jobs, T);
}
void launch_moddown_conv(const DevTables& T, const ModDownJob* jobs, int n_jobs, hipStream_t s) {
  if (n_jobs <= 0) return;
  dim3 grid((1 << T.log_n) / 256, 1, n_jobs);
  hipLaunchKernelGGL(k_moddown_conv, grid, dim3(256), 0, s, jobs, T);
}
void launch_inner(const DevTables& T, const InnerJob* jobs, int n_jobs, int max_ext, hipStream_t s) {
  if (n_jobs <= 0 || max_ext <= 0) return;
  dim3 grid(ew_blocks(1 << T.log_n), n_jobs, max_ext);
  hipLaunchKernelGGL(k_inner, grid, dim3(256), 0, s, jobs, T);
}
void launch_automorph(const DevTables& T, const AutoJob* jobs, int n_jobs, int max_limbs, hipStream_t s) {
  if (n_jobs <= 0 || max_limbs <= 0) return;
  dim3 grid(ew_blocks(1 << T.log_n), max_limbs, n_jobs);
  hipLaunchKernelGGL(k_automorph, grid, dim3(256), 0, s, jobs, T);
}
void launch_lift(const DevTables& T, const LiftJob* jobs, int n_jobs, const double* ctab, double q0inv_q1, hipStream_t s) {
  if (n_jobs <= 0) return;
  dim3 grid((1 << T.log_n) / 256, 1, n_jobs);
  hipLaunchKernelGGL(k_lift, grid, dim3(256), 0, s, jobs, T, ctab, q0inv_q1);
}
void launch_bsgs(const DevTables& T, const BsgsJob* jobs, int n_jobs, int max_limbs, hipStream_t s) {
  if (n_jobs <= 0 || max_limbs <= 0) return;
  dim3 grid(ew_blocks(1 << T.log_n), max_limbs, n_jobs);
  hipLaunchKernelGGL(k_bsgs, grid, dim3(256), 0, s, jobs, T);
}
void launch_raise(const DevTables& T, const RaiseJob* jobs, int n_jobs, hipStream_t s) {
  if (n_jobs <= 0) return;
  dim3 grid((1 << T.log_n) / 256, 1, n_jobs);
  hipLaunchKernelGGL(k_raise, grid, dim3(256), 0, s, jobs, T);
}
void launch_sample(const DevTables& T, const SampleJob* jobs, int n_jobs, int max_limbs, hipStream_t s) {
  if (n_jobs <= 0 || max_limbs <= 0) return;
  dim3 grid(ew_blocks(1 << T.log_n), max_limbs, n_jobs);
  hipLaunchKernelGGL(k_sample, grid, dim3(256), 0, s, jobs, T);
}
void launch_int_spread(const DevTables& T, const IntSpreadJob* jobs, int n_jobs, int max_limbs, hipStream_t s) {
  if (n_jobs <= 0 || max_limbs <= 0) return;
  dim3 grid(ew_blocks(1 << T.log_n), max_limbs, n_jobs);
  hipLaunchKernelGGL(k_int_spread, grid, dim3(256), 0, s, jobs, T);
}
void launch_encode(const DevTables& T, const EncodeJob* jobs, int n_jobs, hipStream_t s) {
  if (n_jobs <= 0) return;
  dim3 grid((1 << T.log_n) / 256, 1, n_jobs);
  hipLaunchKernelGGL(k_encode, grid, dim3(256), 0, s, jobs, T);
}
void launch_fft_enc(const DevTables& T, const FftEncJob* jobs, int n_jobs, int phase, hipStream_t s) {
  if (n_jobs <= 0) return;
  const int N = 1 << T.log_n;
  // zeroing covers 2N elements; scatter covers N/2 slots; stages and rounding N
  const int work = phase == -2 ? 2 * N : phase == -1 ? N / 2 : N;
  dim3 grid((work + 255) / 256, n_jobs, 1);
  hipLaunchKernelGGL(k_fft_enc, grid, dim3(256), 0, s, jobs, T, phase);
}
void launch_decode(const DevTables& T, const int64_t* m, double* z, int nslots, double inv_scale, hipStream_t s) {
  if (nslots <= 0) return;
  hipLaunchKernelGGL(k_decode, dim3(nslots), dim3(256), 0, s, m, z, inv_scale, T);
}

}  // namespace secpe
