// Host tables of the bootstrapping pipeline (boot_tables.cpp, binary128).
#pragma once
#include <stdint.h>

#include <vector>

namespace secpe {

// one generalised diagonal of a slot map: out[p] += (re + i im)[p] in[(p + off) mod ns],
// the vectors of length ns (repeated over the N/2 slots)
struct BootDiag {
  int off = 0;
  std::vector<double> re, im;
};

// a group of merged radix-2 stages: offsets are multiples of delta; baby steps
// 0..n1-1 and giant steps n1 * G cover the centred multiples e in [-E/2, E/2)
struct BootGroupTable {
  int len = 0, delta = 0, n1 = 0, E = 0;
  int ns = 0;   // period of the slot vectors (E = ns / delta)
  std::vector<BootDiag> diags;
};

// stages per group: log2(slots) stages split into 'groups' runs, larger first
int boot_group_len(int log_slots, int groups, int g);
// geometry only (no slot vectors); log_ns = log_n - 1 for the full transforms,
// log2 n for the sparse-slot ones
BootGroupTable boot_group_geometry(int log_n, int log_ns, int groups, int inverse, int g);
// inverse = 1: CoeffToSlot group g (stages m = ns, ns/2, ... in that order),
// scaled by 1 / (2 (K+1)) (and n / (N/2) when sparse) in group 0; inverse =
// 0: SlotToCoeff group g (m = 2, 4, ...), scaled by 2^ratio / (2 pi) in
// group 0.  Sparse: the last CoeffToSlot group writes [w, 0] with period 2n,
// the first SlotToCoeff group transforms a + i b of its input [a, b].
BootGroupTable boot_group_table(int log_n, int log_ns, int groups, int K, int ratio, int inverse, int g);
// Chebyshev coefficients c_0..c_deg of cos(2 pi ((K+1) u - 1/4) / 2^r) on [-1, 1]
void boot_cheb_coeffs(int K, int r, int deg, double* out);

}  // namespace secpe
