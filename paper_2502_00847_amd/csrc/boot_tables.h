// Host tables of the bootstrapping pipeline (boot_tables.cpp, binary128).
#pragma once
#include <stdint.h>

#include <vector>

namespace secpe {

// one generalised diagonal of a slot map: out[p] += (re + i im)[p] in[(p + off) mod S]
struct BootDiag {
  int off = 0;
  std::vector<double> re, im;
};

// a group of merged radix-2 stages: offsets are multiples of delta; baby steps
// 0..n1-1 and giant steps n1 * G cover the centred multiples e in [-E/2, E/2)
struct BootGroupTable {
  int len = 0, delta = 0, n1 = 0, E = 0;
  std::vector<BootDiag> diags;
};

// stages per group: log2(N/2) stages split into 'groups' runs, larger first
int boot_group_len(int log_slots, int groups, int g);
// geometry only (no slot vectors)
BootGroupTable boot_group_geometry(int log_n, int groups, int inverse, int g);
// inverse = 1: CoeffToSlot group g (stages m = S, S/2, ... in that order),
// scaled by 1 / (2 (K+1)) in group 0; inverse = 0: SlotToCoeff group g
// (m = 2, 4, ...), scaled by 2^ratio / (2 pi) in group 0
BootGroupTable boot_group_table(int log_n, int groups, int K, int ratio, int inverse, int g);
// Chebyshev coefficients c_0..c_deg of cos(2 pi ((K+1) u - 1/4) / 2^r) on [-1, 1]
void boot_cheb_coeffs(int K, int r, int deg, double* out);

}  // namespace secpe
