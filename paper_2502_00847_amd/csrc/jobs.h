// Launch descriptors shared by the host runtime and the kernels.
//
// Every kernel is batched: blockIdx.z selects a job (one ciphertext or
// polynomial of one query), blockIdx.y a limb, blockIdx.x a tile of
// coefficients.  Jobs carry their own level, so one launch can mix queries at
// different levels.  Limb l of a polynomial over the basis "n_chain chain
// primes, then special primes" uses prime l when l < n_chain and prime
// n_q + (l - n_chain) otherwise; its coefficients start at data + l * N.
#pragma once
#include <stdint.h>

namespace secpe {

struct DevTables {
  const double* mod;    // [n_mod] primes as doubles
  const double* minv;   // [n_mod] fl(1/p)
  const double* psi;    // [n_mod][N] psi^bitrev(k), forward twiddles
  const double* psiq;   // [n_mod][N] fl(psi/p)
  const double* ipsi;   // [n_mod][N] psi^-bitrev(k), inverse twiddles
  const double* ipsiq;  // [n_mod][N]
  const double* ninv;   // [n_mod] N^-1 mod p
  const double* ninvq;  // [n_mod]
  const double* cos_hi; // [2N] cos(pi t / N) as a double-double (hi, lo)
  const double* cos_lo;
  int n_q, n_p, log_n, pad;
};

enum NttEpi : int {
  EPI_NONE = 0,      // dst = v
  EPI_RESCALE = 1,   // eout = (ea - v) ek[l]
  EPI_RRCOMB = 2,    // eout = (ek2[l] ea + eb - v) ek[l]
  EPI_MODDOWN = 3,   // eout = (ebase or 0) + (eb - v) ek[l]
  EPI_LINRS = 4,     // eout = ([ek2[l] ea + ek3[l] eb] - v) ek[l]   (eb optional; [.] canonical)
};

// NTT over limbs [0, n_limbs) of src (skipping [skip_lo, skip_hi)), written to dst.
// Forward transforms may fuse a prologue into their first pass and an
// epilogue into their last:
//  * spread_from > 0: every limb l reads the one limb at src (coefficient
//    domain, residues mod prime spread_from - 1, taken centred) reduced mod
//    its own prime, instead of limb l of src;
//  * epi != EPI_NONE: the transform v of limb l is not stored; eout at the
//    same position receives the combination above (ea, eb, ebase, eout are
//    limb-major arrays indexed like dst; ek, ek2, ek3 per-limb constants).
//    EPI_LINRS is a constant combination and its rescale in one: the
//    combination is formed here rather than read back from HBM.
//  * sq (squares of degree-1 ciphertexts, two-pass sizes): an inverse
//    transform squares src on load; the EPI_RRCOMB epilogue takes its d as
//    ea^2 (sq = 1) or 2 ea ebase (sq = 2) instead of reading it.
struct NttJob {
  const double* src;
  double* dst;
  int n_limbs, n_chain, skip_lo, skip_hi;
  int spread_from, epi;
  int sq;
  int centre;   // inverse transform: store the last pass centred, in (-p/2, p/2]
  const double* ea;
  const double* eb;
  const double* ebase;
  double* eout;
  const double* ek;
  const double* ek2;
  const double* ek3;
};

enum EwOp : int {
  EW_ADD = 0,        // o0 = a0 + b0, o1 = a1 + b1
  EW_SUB = 1,        // o0 = a0 - b0, o1 = a1 - b1
  EW_TENSOR = 2,     // o0 = a0 b0, o1 = a0 b1 + a1 b0, o2 = a1 b1
  EW_ADD_CONST = 4,  // o0 = a0 + k[l], o1 = a1
  EW_PMUL = 5,       // o_i = a_i * b0 (plaintext polynomial b0)
  EW_DEC2 = 8,       // o0 = a0 + a1 * b0   (b0 = secret key limb)
  EW_ENC = 9,        // o0 = m + e - a s   with a0 = m, a1 = e, b0 = a, b1 = s
  EW_KEYB = 10,      // o0 = e - a s + k[l] s'   with a1 = e, b0 = a, b1 = s, c0 = s'
  EW_MUL = 11,       // o0 = a0 * b0 (single polynomial)
  EW_COPY = 12,      // o0 = a0, o1 = a1
  // degree-2 sum of up to two tensor products plus a degree-1 addend:
  //   o0 = a0 b0 + c0 e0 + f0,  o1 = a0 b1 + a1 b0 + c0 e1 + c1 e0 + f1,  o2 = a1 b1 + c1 e1
  // (c/e and f optional; with k set, f stands for the combination f k + g k2)
  EW_TENSOR2 = 13,
  EW_LIN2 = 15,      // o_i = a_i k[l] + b_i k2[l]   (b optional)
  EW_PADD = 16,      // o0 = a0 + b0 (plaintext polynomial b0), o1 = a1
  EW_PMAC = 17,      // o_i = a_i * b0 + c_i (plaintext product accumulated; c may alias o)
  EW_ADDSUB = 18,    // o0 = a0 - b0, o1 = a0 + b0 (one polynomial: difference and sum from one read)
};

struct EwJob {
  double* o0;
  double* o1;
  double* o2;
  const double* a0;
  const double* a1;
  const double* b0;
  const double* b1;
  const double* c0;
  const double* c1;
  const double* e0;
  const double* e1;
  const double* f0;
  const double* f1;
  const double* k;   // per-limb constants (canonical residues) or null
  const double* k2;  // second per-limb constant table or null
  const double* g0;  // EW_TENSOR2 with k set: the addend is f k[l] + g k2[l] (g optional)
  const double* g1;
  int n_limbs, n_chain;
  int op, l_first;   // limbs below l_first are left untouched
};

// ModUp of one digit: src (coefficient domain, limbs 0..level) -> dst limbs of
// the extended basis Q_level u P outside the digit, coefficient domain.
struct ModUpJob {
  const double* src;
  double* dst;          // [n_ext][N], limb index = extended-basis index
  const double* cinv;   // [digit size] (D/q_i)^-1 mod q_i
  const double* chat;   // [n_ext][digit size] (D/q_i) mod target
  int digit_lo, digit_hi, n_chain, n_ext;
};

// Conv_{B->Q} with centred digits: src = the limbs of B (coefficient domain) ->
// dst chain limbs 0..n_chain-1.  B is the special primes (first_prime < 0) or
// prime first_prime followed by the special primes.  With cinv null, src
// already holds y_b = [x_b (B/b)^-1]_b (the inverse transform's last pass
// scaled by them), canonical or centred.  The column-fused kernel takes it
// centred (NttJob::centre on that pass) and writes dst after the forward
// transform's column pass.
struct ModDownJob {
  const double* src;    // [|B|][N]
  double* dst;          // [n_chain][N]
  const double* cinv;   // [|B|] (B/b)^-1 mod b, or null (see above)
  const double* chat;   // [n_chain][|B|] (B/b) mod q_i
  int n_chain, first_prime;
};

// Inner product with a switching key: acc_w[t] = sum_j x_j[t] * key_j[w][t]
// When top0 is set, limb n_chain-1 of acc_w also gets pmq[n_chain-1] * top_w
// (the top limb of P d_w for the merged relinearise + rescale).
// The fused kernel (N > 2^12) writes limbs t >= inv_from of acc after the
// first pass of their inverse transform (the column pass follows).  With
// d_square set, d (and top) hold a1 (and a0, a1) of a square: the digit
// limbs are d^2 and the top term is a0^2 (w = 0) or 2 a0 a1 (w = 1).
struct InnerJob {
  const double* d;      // NTT-domain input polynomial (chain limbs 0..level)
  const double* ext;    // [dnum][n_ext][N] ModUp outputs, NTT domain
  const double* key;    // [dnum_top][2][n_mod][N]
  double* acc;          // [2][n_ext][N]
  const double* top0;   // optional [n_chain][N], NTT domain
  const double* top1;
  const double* pmq;    // [n_q] P mod q_t
  int n_chain, n_ext, n_digits, alpha;
  int inv_from, d_square;
};

// Galois automorphism in the NTT domain (bit-reversed evaluation order)
struct AutoJob {
  const double* src;
  double* dst;
  int n_limbs, n_chain;
  uint32_t galois, pad;
};

// refresh / encryption: CRT-lift m from limbs 0,1 (coefficient domain) and
// write m mod q_t for t < n_out
struct LiftJob {
  const double* r0;
  const double* r1;
  double* dst;          // [n_out][N]
  int64_t* m_out;       // optional: centred value as int64
  int n_out, pad;
};

// SAMPLE_SPARSE: nonzero (+-1 by the lowest bit) iff the top log2 N bits of
// the draw are below 'param' (the expected Hamming weight h)
enum SampleKind : int { SAMPLE_UNIFORM = 0, SAMPLE_CBD = 1, SAMPLE_TERNARY = 2, SAMPLE_SPARSE = 3 };

struct SampleJob {
  double* dst;          // [n_limbs][N]
  uint64_t seed;
  uint64_t tag_base;    // tag with limb field 0; uniform adds the prime index
  int n_limbs, n_chain, kind, param;
};

// spread an int64 polynomial (host- or device-encoded) to limbs mod q_t
struct IntSpreadJob {
  const int64_t* src;
  double* dst;
  int n_limbs, n_chain;
};

// encode: m_k = round(scale * 2/N * sum_{j < nnz} (z_j cos + zi_j sin)(pi (5^j k mod 2N)/N));
// sparse form (gs set): entry j is slot s_j with gs[j] = 5^{s_j} mod 2N
struct EncodeJob {
  const double* z;      // [nnz] slot values (real parts)
  int64_t* m;           // [N]
  double scale_hi, scale_lo;   // scale * 2 / N as a double-double
  int nnz, pad;
  const uint32_t* gs;   // optional [nnz]
  const double* zi;     // optional [nnz] imaginary parts
};

// Dense complex encoding through one length-2N FFT in double-double (the
// bootstrapping set-up's diagonals, every slot nonzero): the sum that
// EncodeJob forms term by term, sum_j z_j cos(pi g_j k / N) + zi_j sin(pi g_j k / N),
// is Re X[k] of X[k] = sum_t A[t] e^(i pi t k / N) with A[g_j] = z_j - i zi_j
// (the g_j = 5^j mod 2N are distinct) and A zero elsewhere.  buf holds two
// sets of four planes (re hi, re lo, im hi, im lo) of 2N doubles each.
struct FftEncJob {
  const double* z;       // [nnz]
  const double* zi;      // [nnz]
  const uint32_t* gs;    // [nnz]
  double* buf;           // [2][4][2N]
  int64_t* m;            // [N]
  double scale_hi, scale_lo;   // scale * 2 / N as a double-double
  int nnz, pad;
};

// one baby-step giant-step group of a linear transform on one ciphertext:
// out_G = sum_b pt[G * 8 + b] * x_b (both polynomials), for giant index
// G < n_giants and baby step b < n1 (a null pt skips the term); NTT domain
struct BsgsJob {
  const double* x0[8];
  const double* x1[8];
  double* o0[8];
  double* o1[8];
  const double* pt[64];
  int n_limbs, n_giants, n1, pad;
};

// ModRaise: the centred value of a coefficient-domain residue mod q_0
// (src, [N]) reduced mod q_t for t < n_out (dst, [n_out][N])
struct RaiseJob {
  const double* src;
  double* dst;
  int n_out, pad;
};

}  // namespace secpe
