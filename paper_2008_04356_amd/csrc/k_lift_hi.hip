// Instantiations of the BR1 lifting surface kernel for the high degrees (N = 10..15).
#define MORTAR_LIFT_HIGH_DEGREES
#include "k_lift.hip"
