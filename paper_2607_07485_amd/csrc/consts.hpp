// Sizes shared by the host driver and the device code.
#pragma once

namespace lsdd {

// Doubles per tridiagonal row of the inverse-iteration scratch: 64 solving
// lanes x (u0, u1, u2, l, iterate), interleaved by lane, plus 64 pivot bytes.
constexpr int INVIT_SLOTS = 5 * 64 + 8;

}  // namespace lsdd
