// Embedded Runge-Kutta 5(4) pair of Cash & Karp (1990): stage coefficients
// a_sj (j < s), 5th-order weights b5 and 4th-order weights b4.  Included by
// every translation unit that runs Runge-Kutta stages (a copy per unit).
#pragma once

#include <hip/hip_runtime.h>

namespace hm {
namespace {

__constant__ double kA[6][5] = {
    {0, 0, 0, 0, 0},
    {1.0 / 5.0, 0, 0, 0, 0},
    {3.0 / 40.0, 9.0 / 40.0, 0, 0, 0},
    {3.0 / 10.0, -9.0 / 10.0, 6.0 / 5.0, 0, 0},
    {-11.0 / 54.0, 5.0 / 2.0, -70.0 / 27.0, 35.0 / 27.0, 0},
    {1631.0 / 55296.0, 175.0 / 512.0, 575.0 / 13824.0, 44275.0 / 110592.0, 253.0 / 4096.0}};
__constant__ double kB5[6] = {37.0 / 378.0, 0.0, 250.0 / 621.0, 125.0 / 594.0, 0.0, 512.0 / 1771.0};
__constant__ double kB4[6] = {2825.0 / 27648.0, 0.0, 18575.0 / 48384.0, 13525.0 / 55296.0, 277.0 / 14336.0, 0.25};

}  // namespace
}  // namespace hm
