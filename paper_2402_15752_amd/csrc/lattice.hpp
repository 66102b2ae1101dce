// Velocity sets of the GPU library.  Compile-time tables, so that every
// loop over directions unrolls into straight-line code with the velocity
// components and weights folded in as immediates.
//
// D2Q9 and D3Q19 carry the flow set g (and the gradient / Laplacian
// stencils); D2Q9 and D3Q7 carry f, h1 and h2.  Weights are the standard
// ones of the DnQm family the paper cites for its lattices (Sec. IV); D3Q7
// uses w0 = 1/4, w = 1/8, cs^2 = 1/4.
#pragma once

namespace pflb {

struct D2Q9 {
  static constexpr int Q = 9;
  static constexpr int D = 2;
  // rest, +x, +y, -x, -y, then the four diagonals
  static constexpr int cx[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
  static constexpr int cy[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
  static constexpr int cz[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
  static constexpr int opp[9] = {0, 3, 4, 1, 2, 7, 8, 5, 6};
  static constexpr double w[9] = {4.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9,
                                  1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36};
  static constexpr double cs2 = 1.0 / 3.0;
};

struct D3Q7 {
  static constexpr int Q = 7;
  static constexpr int D = 3;
  static constexpr int cx[7] = {0, 1, -1, 0, 0, 0, 0};
  static constexpr int cy[7] = {0, 0, 0, 1, -1, 0, 0};
  static constexpr int cz[7] = {0, 0, 0, 0, 0, 1, -1};
  static constexpr int opp[7] = {0, 2, 1, 4, 3, 6, 5};
  static constexpr double w[7] = {0.25, 0.125, 0.125, 0.125, 0.125, 0.125, 0.125};
  static constexpr double cs2 = 0.25;
};

struct D3Q19 {
  static constexpr int Q = 19;
  static constexpr int D = 3;
  // rest, 6 axis links, then the 12 edge links grouped by plane (xy, xz, yz)
  static constexpr int cx[19] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
  static constexpr int cy[19] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1};
  static constexpr int cz[19] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1};
  static constexpr int opp[19] = {0, 2, 1, 4, 3, 6, 5, 8, 7, 10, 9, 12, 11, 14, 13, 16, 15, 18, 17};
  static constexpr double w[19] = {1.0 / 3,  1.0 / 18, 1.0 / 18, 1.0 / 18, 1.0 / 18,
                                   1.0 / 18, 1.0 / 18, 1.0 / 36, 1.0 / 36, 1.0 / 36,
                                   1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36,
                                   1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36};
  static constexpr double cs2 = 1.0 / 3.0;
};

// Population planes in a lattice buffer: f, g, h1, h2 back to back.
template <class LF, class LG>
struct Layout {
  static constexpr int QF = LF::Q;
  static constexpr int QG = LG::Q;
  static constexpr int F0 = 0;
  static constexpr int G0 = QF;
  static constexpr int H10 = QF + QG;
  static constexpr int H20 = 2 * QF + QG;
  static constexpr int QTOT = 3 * QF + QG;
};

}  // namespace pflb
