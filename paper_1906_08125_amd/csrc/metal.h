// Metal-side solves (Sec. II D, App. C-D): mesh setup, continuity solve
// with Joule heating, and one Theta-scheme heat step.  The C ABI wrappers
// check arguments; these calls report errors through *err.
#pragma once
#include <string>

#include "common.h"

namespace fp {

pic_status metal_build(const pic_metal_desc* d, hipStream_t s, pic_metal** out,
                       std::string* err);
void metal_free(pic_metal* h);
int64_t metal_n_faces(const pic_metal* h);
pic_status metal_continuity(pic_metal* h, const double* sigma, const double* flux,
                            double tol, int64_t max_iter, double* phi, double* pj,
                            pic_metal_stats* st, hipStream_t s, std::string* err);
pic_status metal_heat(pic_metal* h, const pic_heat_params* p, const double* sigma,
                      const double* pj, const double* pn, double* T,
                      pic_metal_stats* st, hipStream_t s, std::string* err);

}  // namespace fp
