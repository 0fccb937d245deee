// Learned cost model (MLP 4 -> 64 -> 64 -> 1, FP32) used only to order and
// bin K-block work units; it never decides culling.
#pragma once
#include <stdint.h>
