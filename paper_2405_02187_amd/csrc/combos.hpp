// Supported (precision, directions D, Hessian size Q) shapes, one translation
// unit each (inst.hip compiled once per line).
#pragma once
#define XS_COMBOS(X)              \
  X(double, 0, 0, c128_d0_q0)     \
  X(double, 1, 0, c128_d1_q0)     \
  X(double, 2, 2, c128_d2_q2)     \
  X(double, 6, 0, c128_d6_q0)     \
  X(float, 0, 0, c64_d0_q0)       \
  X(float, 1, 0, c64_d1_q0)       \
  X(float, 2, 0, c64_d2_q0)       \
  X(float, 2, 2, c64_d2_q2)       \
  X(float, 3, 0, c64_d3_q0)       \
  X(float, 4, 0, c64_d4_q0)       \
  X(float, 4, 4, c64_d4_q4)       \
  X(float, 5, 0, c64_d5_q0)       \
  X(float, 6, 0, c64_d6_q0)       \
  X(float, 16, 0, c64_d16_q0)     \
  X(float, 16, 4, c64_d16_q4)
