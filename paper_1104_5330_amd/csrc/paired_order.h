// Paired in-plane order of the stage buffers on the 32 x 64 position sphere:
// within every Theta row of n_Phi values, g consecutive Phi of the first half are
// followed by the g at Phi + pi, so that a fused theta-phi tile (those 2 g
// columns, closed under the partner map of the theta lines) is one run instead of
// two: g = 4 for the FP64 state (tiles of eight FP64 columns, 64-byte runs),
// g = 8 for the FP32 stage copy of the mixed path (tiles of sixteen FP32
// columns, 64-byte runs).  Column Phi of a row with hP = n_Phi / 2 (a multiple of
// g) sits at
//   2 g ((Phi mod hP) div g) + g [Phi >= hP] + Phi mod g.
// The permutation stays inside each row, so Theta-dependent factors (radial
// coefficient, inflow nodes) and every per-plane quantity are unchanged.
// Plain constexpr functions (callable from device code too); the host-only
// unit test builds this header on its own.
#pragma once

constexpr int paired_pos(int phi, int hP, int g = 4) {
  return 2 * g * ((phi >= hP ? phi - hP : phi) / g) + g * (phi >= hP ? 1 : 0) + (phi >= hP ? phi - hP : phi) % g;
}
// its inverse: the column Phi stored at position pos of a row
constexpr int paired_phi(int pos, int hP, int g = 4) { return g * (pos / (2 * g)) + pos % g + ((pos / g) & 1) * hP; }
