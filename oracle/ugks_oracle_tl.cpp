/*
 * Tangent build of the oracle: ugks_oracle.c compiled as C++ with the scalar
 * type set to the forward-mode dual number of or_dual.h.
 *
 * TEST INFRASTRUCTURE ONLY.  Every entry point of ugks_oracle.h is exported
 * with the same name and the same arguments, each real being a (value,
 * tangent) pair of doubles; the results carry the directional derivative of
 * the method along the seeded input tangents.  This is the reference gradient
 * that the hand-written adjoint of the HIP library is checked against.
 */
#define OR_TANGENT 1
#include "ugks_oracle.c"
