// Paired in-plane order of the FP64 stage buffers on the 32 x 64 position sphere
// (RK stages 2 to 4): within every Theta row of n_Phi values, four consecutive
// Phi of the first half are followed by the four at Phi + pi, so that a fused
// theta-phi tile (those eight columns, closed under the partner map of the theta
// lines) is one 64-byte run instead of two 32-byte runs.  Column Phi of a row
// with hP = n_Phi / 2 (a multiple of 4) sits at
//   8 ((Phi mod hP) div 4) + 4 [Phi >= hP] + Phi mod 4.
// The permutation stays inside each row, so Theta-dependent factors (radial
// coefficient, inflow nodes) and every per-plane quantity are unchanged.
// Plain constexpr functions (callable from device code too); the host-only
// unit test builds this header on its own.
#pragma once

constexpr int paired_pos(int phi, int hP) {
  return 8 * ((phi >= hP ? phi - hP : phi) >> 2) + 4 * (phi >= hP ? 1 : 0) + ((phi >= hP ? phi - hP : phi) & 3);
}
// its inverse: the column Phi stored at position pos of a row
constexpr int paired_phi(int pos, int hP) { return 4 * (pos >> 3) + (pos & 3) + ((pos >> 2) & 1) * hP; }
