// Sizes shared by the host driver and the device code.
#pragma once

namespace lsdd {

// Doubles per tridiagonal row of the inverse-iteration scratch: 64 solving
// lanes x (u0, u1, u2, iterate), interleaved by lane.
constexpr int INVIT_SLOTS = 4 * 64;

}  // namespace lsdd
