// Exact RNS modular arithmetic in IEEE binary64 for gfx950.
//
// Every residue is an integer held exactly in a double.  All moduli are odd
// primes p < 2^51.  CDNA4 issues FP64 FMA at the full vector rate, so a
// modular product costs six FP64 instructions here, against roughly twenty
// (ten of them 32-bit multiplies) for the 64-bit integer Shoup/Barrett form.
//
// mul_w(a, w, wq, p): Barrett reduction with a floating-point quotient.
//   hi + lo = a*w exactly (FMA two-product, Dekker 1971 / Ogita-Rump-Oishi 2005);
//   q = rint(a * wq) with wq = fl(w/p) is within 1.65 of a*w/p for |a| < 2.3p;
//   r = (hi - q p) + lo is then an integer below 2^53 in magnitude, so the FMA
//   and the add are exact.  Result: r = a*w (mod p), |r| < 1.7p.
// red(x): x - p * rint(x/p) for |x| < 2^53, exact, |result| <= p/2 + 1.
//
// Values in registers are signed and lazily reduced; everything stored to HBM
// is canonical, in [0, p).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace secpe {

struct Mod {
  double p;     // prime
  double pinv;  // fl(1/p)
};

__device__ __forceinline__ double fma_rn(double a, double b, double c) { return __builtin_fma(a, b, c); }

// |a| < 2^52.2 (about 2.3p), 0 <= w < p, wq = fl(w/p)  ->  |result| < 1.7p, == a*w mod p
__device__ __forceinline__ double mul_w(double a, double w, double wq, double p) {
  double hi = a * w;
  double lo = fma_rn(a, w, -hi);
  double q = __builtin_rint(a * wq);
  double r = fma_rn(-q, p, hi);
  return r + lo;
}

// general product, |a|,|b| < p  ->  |result| < 1.3p
__device__ __forceinline__ double mul_mod(double a, double b, const Mod& m) {
  double hi = a * b;
  double lo = fma_rn(a, b, -hi);
  double q = __builtin_rint(hi * m.pinv);
  double r = fma_rn(-q, m.p, hi);
  return r + lo;
}

// |x| < 2^53  ->  |result| <= p/2 + 1
__device__ __forceinline__ double red(double x, const Mod& m) {
  double q = __builtin_rint(x * m.pinv);
  return fma_rn(-q, m.p, x);
}

// |x| < 2^53  ->  canonical in [0, p)
__device__ __forceinline__ double canon(double x, const Mod& m) {
  double r = red(x, m);
  return r < 0.0 ? r + m.p : r;
}

// |x| < 2p -> canonical (one-step correction for values already near range)
__device__ __forceinline__ double canon_small(double x, const Mod& m) {
  double r = x < 0.0 ? x + m.p : x;
  return r >= m.p ? r - m.p : r;
}

__device__ __forceinline__ double add_mod(double a, double b, const Mod& m) {  // a, b canonical
  double s = a + b;
  return s >= m.p ? s - m.p : s;
}
__device__ __forceinline__ double sub_mod(double a, double b, const Mod& m) {  // a, b canonical
  double s = a - b;
  return s < 0.0 ? s + m.p : s;
}

// Pointers read from job descriptors are generic; casting them to the global
// address space lets the compiler emit global_load / global_store.
typedef __attribute__((address_space(1))) double gdbl;
typedef const __attribute__((address_space(1))) double cgdbl;
#define GPTR(p) ((gdbl*)(p))
#define CGPTR(p) ((cgdbl*)(p))
// read-only tables: the constant address space lets uniform indices become
// scalar loads
typedef const __attribute__((address_space(4))) double kdbl;
#define KPTR(p) ((kdbl*)(p))
typedef double dv2 __attribute__((ext_vector_type(2)));
typedef __attribute__((address_space(1))) dv2 gdbl2;
typedef const __attribute__((address_space(1))) dv2 cgdbl2;

// uint64 <-> double for values below 2^53
__device__ __forceinline__ double u64_to_d(uint64_t v) { return (double)v; }
__device__ __forceinline__ uint64_t d_to_u64(double v) { return (uint64_t)v; }

}  // namespace secpe
