// Host runtime: context, device tables, command lists and batched CKKS ops.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <map>
#include <string>
#include <vector>

#include "kernels.h"

namespace secpe {

using u128 = unsigned __int128;

// ---------------------------------------------------------------------------
// host modular arithmetic for table construction
// ---------------------------------------------------------------------------
inline uint64_t hmul(uint64_t a, uint64_t b, uint64_t q) { return (uint64_t)((u128)a * b % q); }
inline uint64_t hpow(uint64_t a, uint64_t e, uint64_t q) {
  uint64_t r = 1 % q;
  a %= q;
  for (; e; e >>= 1) {
    if (e & 1) r = hmul(r, a, q);
    a = hmul(a, a, q);
  }
  return r;
}
inline uint64_t hinv(uint64_t a, uint64_t q) { return hpow(a % q, q - 2, q); }
inline uint64_t hmod_i64(int64_t v, uint64_t q) {
  int64_t r = v % (int64_t)q;
  return (uint64_t)(r < 0 ? r + (int64_t)q : r);
}

// ---------------------------------------------------------------------------
// context
// ---------------------------------------------------------------------------
struct DigitTable {
  const double* cinv;  // [dsz]
  const double* chat;  // [n_mod][dsz], indexed by absolute prime
};

struct KeyRef {
  const double* base;  // [dnum][2][n_mod][N]
};

struct Ctx;

// one group of a bootstrapping linear transform, its plaintexts precomputed:
// diagonal i (slot offset off[i] = delta e, e centred) is stored pre-rotated by
// -delta n1 floor(e / n1) and encoded for an input of scale in_scale at 'level'
struct BootGroup {
  int inverse = 0, g = 0, level = 0, delta = 0, n1 = 0, E = 0;
  int log_ns = 0;                  // log2 of the transform's slot count (N/2 or the sparse n)
  double in_scale = 0.0, pscale = 0.0, out_scale = 0.0;
  std::vector<int64_t> e;          // centred offset multiple of each diagonal
  std::vector<const double*> pt;   // NTT domain, limbs 0..level
};

// the step value that asks for the conjugation X -> X^(2N-1)
constexpr int64_t kConjStep = INT64_MIN;

struct GraphEntry {
  uint64_t hash = 0;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  char* arena = nullptr;
  size_t arena_bytes = 0;
  std::vector<int> out_level;
  std::vector<double> out_scale;
  int64_t counters[8] = {0};
  int64_t ks_alg_limbs = 0;
};

struct Ctx {
  // parameters
  int log_n = 0, N = 0, n_q = 0, n_p = 0, alpha = 0, dnum = 0, n_mod = 0;
  // two-pass NTT launches are issued in job groups of at most this many bytes
  // of limb data (0 = one group); SECPE_NTT_CHUNK_MB overrides the default
  size_t ntt_chunk_bytes = 0;
  // output limbs per workgroup of the column-fused base conversions, ModUp
  // and ModDown (2 or 4 each); set by the autotuner
  int modup_eg = 4, moddown_eg = 4;
  // NTT passes with two tiles per workgroup (bit 0 forward column, bit 1
  // inverse column, bit 2 forward row); set by the autotuner
  int ntt_tiles = 0;
  int q_bits = 0, p_bits = 0, log_scale = 0, dg = 2, df = 2, min_level = 1;
  int refresh_level = 0;   // level a refreshed ciphertext is re-encrypted at
  int refresh_level_set = 0;  // the level the parameters asked for (bootstrapping may override it)
  // bootstrapping (secpe_set_boot, secpe_boot_setup)
  int secret_h = 0;        // > 0: sparse secret of expected Hamming weight h
  int boot_mode = 0;       // 1: refreshes are bootstraps
  int boot_K = 0, boot_r = 0, boot_deg = 0, boot_ratio = 0, boot_groups = 0;
  int boot_out_level = -1;
  std::vector<double> boot_cheb;
  std::vector<BootGroup> boot_cts, boot_stc;   // CoeffToSlot, SlotToCoeff groups
  int boot_sparse = 0;     // n > 0: the sparse-slot bootstrap keeps slots [0, n)
  std::vector<BootGroup> boot_cts_sp, boot_stc_sp;   // its transforms
  const double* boot_mono = nullptr;            // X^(N/2), then -X^(N/2): [2][n_q][N], NTT domain
  bool boot_ready = false;
  int boot_chunk = 8;      // ciphertexts bootstrapped together in one pass
  // k >= 2: a refresh of at least k ciphertexts that read only slots
  // [0, boot_sparse) again packs them into shared full-slot bootstraps
  int boot_pack_min = 0;
  std::vector<uint64_t> mod;
  int device = 0;
  hipStream_t stream = nullptr;
  // device tables
  double* d_tab = nullptr;
  size_t tab_bytes = 0;
  DevTables T{};
  std::map<std::pair<int, int>, DigitTable> digits;  // (digit_lo, size)
  const double* md_cinv = nullptr;   // [alpha]
  const double* md_chat = nullptr;   // [n_q][alpha]
  const double* md_pinv = nullptr;   // [n_q] P^-1 mod q_t
  const double* p_mod_q = nullptr;   // [n_q] P mod q_t
  const double* rs_tab = nullptr;    // [n_q][n_q] q_l^-1 mod q_i at [l][i]
  const double* ytab = nullptr;      // [n_q][n_q] N^-1 (D_j/q_t)^-1 mod q_t at [l][t]
  // merged relinearise + rescale at level l over B = {q_l} u P
  const double* rr_cinv = nullptr;   // [n_q][alpha+1] (B/b)^-1 mod b
  const double* rr_chat = nullptr;   // [n_q][n_q][alpha+1] (B/b) mod q_t
  const double* rr_inv = nullptr;    // [n_q][n_q] (P q_l)^-1 mod q_t
  // the inverse transform feeding a conversion from B scales limb b by
  // N^-1 (B/b)^-1 mod b: B = P at [k] (special prime k), B = {q_l} u P at
  // [l][l + i] (i = 0: q_l; i = 1 + k: special prime k)
  const double* md_ytab = nullptr;   // [alpha]
  const double* rr_ytab = nullptr;   // [n_q][n_q + alpha]
  const double* crt_tab = nullptr;   // [n_q][2]
  double q0inv_q1 = 0.0;
  // keys
  std::map<uint64_t, const double*> keys;  // Galois element -> key; 0 = relinearisation
  // Galois element g -> its key with every limb taken through X -> X^(g^-1)
  // (NTT-domain permutation), for the hoisted baby steps of the sparse-slot
  // transforms; built by secpe_boot_setup in its buffer, cleared with the keys
  std::map<uint64_t, const double*> keys_perm;
  // descriptor arena
  char* arena = nullptr;
  size_t arena_bytes = 0;
  char* staging = nullptr;  // pinned
  size_t staging_bytes = 0;
  hipEvent_t staging_done = nullptr;
  // client scratch
  char* client = nullptr;
  size_t client_bytes = 0;
  // statistics of the last evaluation
  int64_t counters[8] = {0};
  // event profiler
  int prof_kind = -1;
  std::vector<hipEvent_t> prof_pool;
  size_t prof_used = 0;
  int64_t prof_launches = 0, prof_units = 0, prof_units_shared = 0;
  std::vector<double> seg_ms;   // intervals of the last segment profile
  // algorithmic HBM limbs of the last evaluation's key switches: per key
  // switch at l+1 limbs, (l+1) read + 2 (l+1) written, plus the key's
  // 2 dnum_l (l+1+alpha) limbs once per launch for all the jobs sharing it
  int64_t ks_alg_limbs = 0;
  std::vector<GraphEntry> graphs;

  size_t limb_bytes() const { return (size_t)N * sizeof(double); }
  size_t ct_bytes() const { return 2 * (size_t)n_q * limb_bytes(); }
  size_t key_bytes() const { return (size_t)dnum * 2 * n_mod * limb_bytes(); }
  size_t sk_bytes() const { return (size_t)n_mod * limb_bytes(); }
  uint64_t galois(int64_t step) const;
};

int build_context(Ctx& c, int log_n, int n_q, int q_bits, int n_p, int p_bits, int log_scale, int dg, int df,
                  int min_level, int refresh_level, int device, hipStream_t stream);
void destroy_context(Ctx& c);
// destroy every captured graph (their launches bake in keys and schedule settings)
void drop_graphs(Ctx& c);

// ---------------------------------------------------------------------------
// command list: descriptors in one blob, launches replayed in order
// ---------------------------------------------------------------------------
enum CmdKind { C_NTT, C_NTT_FIRST, C_NTT_SECOND, C_EW, C_MODUP, C_MODUP_COL, C_MODDOWN, C_MODDOWN_COL, C_INNER, C_INNER_ROW, C_AUTO, C_LIFT, C_SAMPLE, C_INTSPREAD, C_ENCODE, C_DECODE, C_RAISE, C_BSGS, C_FFTENC,
               C_MARK /* no launch: a segment boundary for the segment profiler */ };

struct Cmd {
  int kind;
  int n;
  int max_y;
  size_t off;
  bool inv;
  const int64_t* m;
  double* z;
  double inv_scale;
  int64_t units;   // limbs processed by the launch (limb transforms for the NTT)
  // the same with data that several jobs of the launch read counted once
  // (the key limbs of the inner product); equals units for the other kinds
  int64_t units_shared;
};

// kinds the event profiler can bracket (secpe_profile_begin)
enum ProfKind { PROF_NTT_FWD = 0, PROF_NTT_INV = 1, PROF_EW = 2, PROF_MODUP = 3, PROF_MODDOWN = 4, PROF_INNER = 5,
                PROF_AUTO = 6, PROF_SPREAD = 7, PROF_NTT_FWD_COL = 8, PROF_NTT_FWD_ROW = 9, PROF_SEGMENTS = 10,
                PROF_NKINDS = 11 };

// ciphertext handle inside a build: device data [2][n_q][N], level, scale, pool slot
struct CT {
  double* d = nullptr;
  int level = -1;
  double scale = 0.0;
  int slot = -1;   // -1: not owned by the pool
};

// ciphertext slots of a workspace; a server keeps one across rounds
struct SlotPool {
  std::vector<int> free_slots;
  int n_slots = 0;   // high-water mark
  int live = 0;
};

class Builder {
 public:
  Builder(Ctx& c, char* ws, size_t ws_bytes, char* arena, size_t arena_bytes, bool dry, SlotPool* pool = nullptr);

  Ctx& C;
  bool dry;
  std::string err;
  int err_code = 0;
  // the key owner's secret for the refresh stand-in of bootstrapping, given
  // per evaluation (never held by the context); null: no refresh available
  const double* refresh_sk = nullptr;

  // memory
  CT new_ct(int level, double scale);
  void free_ct(CT& x);
  double* scratch(size_t n_doubles);
  size_t scratch_mark() const { return scratch_cur_; }
  void scratch_release(size_t mark) { scratch_cur_ = mark; }
  size_t need_bytes() const { return need_max_; }
  int peak_slots() const { return peak_live_; }
  size_t peak_scratch() const { return peak_scratch_; }
  size_t blob_bytes() const { return blob_.size(); }
  bool arena_overflow() const { return blob_.size() > arena_bytes_; }

  double* c0(const CT& x) const { return x.d; }
  double* c1(const CT& x) const { return x.d + (size_t)C.n_q * C.N; }

  // descriptor / constant uploads (returns device addresses inside the arena)
  template <class J>
  const J* put(const std::vector<J>& v) {
    return (const J*)put_bytes(v.data(), v.size() * sizeof(J));
  }
  const void* put_bytes(const void* p, size_t n);
  const double* put_residues(int64_t K, int n_limbs);  // K mod q_t, t < n_limbs (chain)

  // raw launches
  // first_pass_only: the column pass of a two-pass forward NTT (its row pass
  // runs inside the fused inner product)
  // pass: -1 = the whole transform; 0 or 1 = only that pass of a two-pass
  // NTT (the other pass runs fused into a neighbouring kernel)
  void ntt(const std::vector<NttJob>& v, bool inverse, int pass = -1);
  void ew(const std::vector<EwJob>& v);
  void modup(const std::vector<ModUpJob>& v);
  void modup_col(const std::vector<ModUpJob>& v);
  void moddown(const std::vector<ModDownJob>& v);
  void moddown_col(const std::vector<ModDownJob>& v);
  // row_fused: with the two-pass NTT, the inner product runs the ext limbs'
  // row pass (their inputs leave the ModUp after the column pass)
  void inner(const std::vector<InnerJob>& v, bool row_fused = true);
  void automorph(const std::vector<AutoJob>& v);
  void lift(const std::vector<LiftJob>& v);
  void raise(const std::vector<RaiseJob>& v);
  void bsgs(const std::vector<BsgsJob>& v);
  void sample(const std::vector<SampleJob>& v);
  void intspread(const std::vector<IntSpreadJob>& v);
  void encode(const std::vector<EncodeJob>& v);
  // dense encodings through a length-2N FFT (max_y of each command = its phase)
  void fft_encode(const std::vector<FftEncJob>& v);
  void decode(const int64_t* m, double* z, int nslots, double inv_scale);
  // a segment boundary (the refresh stand-in marks its start and end)
  void mark();

  // CKKS operations over batches of items
  struct KsItem {
    const double* d;      // NTT domain, chain limbs 0..level
    int level;
    const double* key;
    const double* base0;  // may be null
    const double* base1;
    double* out0;
    double* out1;
    const double* top0;   // merged relinearise + rescale: d0, d1 (else null)
    const double* top1;
    bool square;          // d, top0, top1 are a1, a0, a1 of a square (fused path)
  };
  struct KsTmp {
    double* dcoef;
    double* ext;
    double* acc;
    int n_ext;
  };
  // degree-2 ciphertext d0 + d1 s + d2 s^2 in scratch, NTT domain; or, when
  // sq0 is set (two-pass sizes), the square of (sq0, sq1) formed on the fly
  // by the kernels that read it
  struct Deg2 {
    double* d0;
    double* d1;
    double* d2;
    int level;
    double scale;
    const double* sq0 = nullptr;
    const double* sq1 = nullptr;
  };
  struct LinItem {
    CT a, b;
    double va, vb, target;
    bool has_b;
  };
  // has_fl: the degree-1 addend is the (unrescaled) constant combination fl,
  // formed inside the degree-2 sum instead of being written out first
  struct TensorItem {
    CT a, b, c, e, f;
    bool has_ce, has_f;
    LinItem fl{};
    bool has_fl = false;
  };
  // merged: the conversion that follows reads limbs level .. level+n_p of the
  // accumulator (merged relinearise + rescale), else the special limbs only;
  // the fused inner product runs the first inverse NTT pass on those limbs
  void ks_front(const std::vector<KsItem>& items, std::vector<KsTmp>& tmp, bool merged);
  void key_switch(const std::vector<KsItem>& items);
  // second half: ModDown by P of each accumulator, added to the item's base;
  // first_pass_done: the inner product already ran the first inverse NTT pass
  void ks_back(const std::vector<KsItem>& items, const std::vector<KsTmp>& tmp, bool first_pass_done);
  // hoisted rotations: the ModUp of each input's c1 once (ext, NTT domain,
  // in scratch until the caller releases it), then rotations of every input
  // by any steps, each applying X -> X^g to the raised digits (or, for a step
  // with a permuted key, to the two results after the ModDown)
  struct Hoisted {
    std::vector<CT> in;
    std::vector<double*> ext;
  };
  Hoisted hoist(const std::vector<CT>& in);
  // out[s * n + i] = RotL(in[i], steps[s])
  std::vector<CT> rotate_hoisted(const Hoisted& h, const std::vector<int64_t>& steps);
  std::vector<Deg2> tensor2(const std::vector<TensorItem>& v);
  std::vector<CT> relin_rescale(const std::vector<Deg2>& xs);
  std::vector<CT> lincomb(const std::vector<LinItem>& v, bool do_rescale);
  void rescale(std::vector<CT>& in_out);                    // in place
  // the sources of a constant combination whose rescale forms it in its
  // epilogue (only the top limb of the combination is in HBM beforehand)
  struct LinSrc {
    const double* a0;
    const double* a1;
    const double* b0;   // null without a second term
    const double* b1;
    const double* ka;   // per-limb residues of the constants
    const double* kb;
  };
  void rescale(std::vector<CT>& in_out, const std::vector<LinSrc>* lin);
  std::vector<CT> mul_relin(const std::vector<std::pair<CT, CT>>& ab, bool do_rescale);
  std::vector<CT> rotate(const std::vector<CT>& in, const std::vector<int64_t>& steps);
  std::vector<CT> add(const std::vector<std::pair<CT, CT>>& ab, bool sub);
  // a - b and a + b of each pair from one read of a and b
  void add_sub(const std::vector<std::pair<CT, CT>>& ab, std::vector<CT>& diff, std::vector<CT>& sum);
  std::vector<CT> add_const(const std::vector<CT>& in, const std::vector<double>& v);
  std::vector<CT> mul_const(const std::vector<CT>& in, const std::vector<double>& v, const std::vector<double>& target);
  std::vector<CT> mul_plain(const std::vector<CT>& in, const std::vector<std::vector<double>>& z,
                            const std::vector<double>& target);
  // slot values given as (slot, value) pairs
  struct SparseSlots {
    std::vector<int> slot;
    std::vector<double> val;
  };
  std::vector<CT> mul_plain_sparse(const std::vector<CT>& in, const std::vector<SparseSlots>& z,
                                   const std::vector<double>& target);
  // x + encode(z) at x's scale
  std::vector<CT> add_plain_sparse(const std::vector<CT>& in, const std::vector<SparseSlots>& z);
  std::vector<CT> plain_op(const std::vector<CT>& in, const std::vector<std::vector<double>>* dense,
                           const std::vector<SparseSlots>* sparse, const std::vector<double>* target, bool product);
  // span[i] > 0: only slots [0, span[i]) of item i are read again (a
  // bootstrap may then keep just those); null: every slot
  std::vector<CT> refresh(const std::vector<CT>& in, const std::vector<uint64_t>& seed,
                          const std::vector<uint64_t>& index, const std::vector<int>* span = nullptr);
  std::vector<CT> eval_odd9(const std::vector<CT>& x, const std::vector<const double*>& coef,
                            const std::vector<double>& gain, const std::vector<double>& target);
  // bootstrapping steps (the groups' plaintexts come from secpe_boot_setup)
  std::vector<CT> mod_raise(const std::vector<CT>& in);                 // level 0 -> top, scale q_0
  std::vector<CT> mul_monomial_half(const std::vector<CT>& in, bool neg);  // slots times +-i
  // sparse: the sparse-slot transforms (the last CoeffToSlot group writes
  // period 2n, the first SlotToCoeff group reads it)
  std::vector<CT> boot_transform(const std::vector<CT>& in, bool inverse, bool sparse = false);
  std::vector<CT> eval_mod(const std::vector<CT>& u);
  std::vector<CT> relin(const std::vector<Deg2>& xs);        // relinearise, no rescale
  void cheb_basis_step(std::vector<std::vector<CT>>& T, std::vector<std::vector<CT>>& T2, int j);
  std::vector<CT> cheb_combination(const std::vector<std::vector<CT>>& T, const double* cf, int nt, int lv,
                                   const std::vector<double>& scale);
  std::vector<CT> cheb_node(const std::vector<std::vector<CT>>& T, int B, int lb, const double* cf, int m,
                            const std::vector<double>& target);
  std::vector<CT> square_exact(const std::vector<CT>& xs);   // relinearise, then rescale
  // sparse: keep slots [0, boot_sparse), repeated with period boot_sparse
  std::vector<CT> bootstrap(const std::vector<CT>& in, bool sparse = false);
  std::vector<CT> bootstrap_chunk(const std::vector<CT>& in);
  std::vector<CT> bootstrap_sparse_chunk(const std::vector<CT>& in);
  // the full pipeline after the scale-down (level-0 inputs at scale
  // q_0 / 2^ratio); frees its inputs
  std::vector<CT> boot_core_full(std::vector<CT> x0);
  // inputs read only on slots [0, W) again (W = boot_sparse), N/2W per
  // shared full-slot bootstrap: output j holds input j's window at [0, W)
  std::vector<CT> bootstrap_packed(const std::vector<CT>& in);
  // x + RotL(x, n) + RotL(x, 2n) + ... over the multiples of n below N/2
  std::vector<CT> subsum(const std::vector<CT>& in, int n);
  // client-side helpers
  void encrypt_into(const std::vector<const int64_t*>& m_dev, const std::vector<uint64_t>& seed, int purpose,
                    const std::vector<uint64_t>& sub, const double* sk, const std::vector<CT>& out);

  void fail(int code, const std::string& msg) {
    if (!err_code) { err_code = code; err = msg; }
  }

  std::vector<char> blob_;
  std::vector<Cmd> cmds_;
  int64_t counters[8] = {0};
  int64_t ks_alg_limbs = 0;   // see Ctx::ks_alg_limbs

 private:
  char* ws_;
  size_t ws_bytes_;
  char* arena_;
  size_t arena_bytes_;
  size_t slot_bytes_;
  SlotPool own_pool_;
  SlotPool* pool_;
  int peak_live_ = 0;
  size_t scratch_cur_ = 0;
  size_t peak_scratch_ = 0;
  size_t need_max_ = 0;
  void note_need();
  void push(int kind, int n, int max_y, size_t off, bool inv = false, int64_t units = 0, int64_t units_shared = -1);
};

// Submit a command list: upload the descriptor blob to 'arena' and launch all
// commands in order on the context's stream.  may_allocate = false: the blob
// goes through the existing pinned staging buffer, never a larger new one
// (-2 when it does not fit).
int submit(Ctx& c, Builder& b, char* arena, size_t arena_bytes, bool may_allocate = true);
void launch_cmds(Ctx& c, const std::vector<Cmd>& cmds, char* arena);
int prof_kind_of(const Cmd& k);

// the encrypted Argmax program over a batch of queries
struct ArgmaxQuery {
  CT in;
  int K, C;
  double d_min, d_max;
  uint64_t refresh_seed;
  CT out;  // caller buffer (d set), level/scale written
  uint64_t ticket = 0;
  // slot-packed input (several Argmax inputs in one ciphertext): per block
  // K, C and the bounds of Eq. 5; empty for one query per ciphertext
  std::vector<int> bK, bC;
  std::vector<double> blo, bhi;
};
// K', C' and block size of a packed group (the largest padded shape; blocks
// of max(K'C', 2C') slots)
void packed_shape(const std::vector<int>& K, const std::vector<int>& C, int* kp, int* cp, int* bsz);
void build_argmax(Builder& b, std::vector<ArgmaxQuery>& q);
// the comparison path (Phoenix) for one query
void build_phoenix(Builder& b, ArgmaxQuery& q);

// Per-query state machines that survive across command lists: a round
// advances queries by one step (all step kinds present, or only the most
// common one) and returns the queries that finished in it.
struct QState;
class ArgmaxProgram {
 public:
  ArgmaxProgram();
  ~ArgmaxProgram();
  bool add(Builder& b, ArgmaxQuery* q);
  std::vector<ArgmaxQuery*> round(Builder& b, bool all_kinds);
  size_t active() const;

 private:
  std::vector<QState*> st_;
};

int ilog2_ceil(int v);

}  // namespace secpe
