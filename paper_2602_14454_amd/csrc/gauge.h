// Quenched gauge-field generation (gauge.hip).
#pragma once

#include <hip/hip_runtime.h>

namespace dwf {

// One sweep over every link of a canonical complex128 field U[lex][mu][3][3]
// (device): heatbath (heatbath = true, random numbers keyed by seed and
// sweep_index) or over-relaxation, then re-projection onto SU(3).
void gauge_sweep(void* U, const int dims[4], double beta, unsigned long long seed, long long sweep_index,
                 bool heatbath, hipStream_t st);
// average Re tr U_P / 3 (FP64 reduction); partial: device scratch of
// gauge_plaquette_partials(dims) + 1 doubles
int gauge_plaquette_partials(const int dims[4]);
void gauge_plaquette(const void* U, const int dims[4], double* partial, double* out_dev, hipStream_t st);

}  // namespace dwf
