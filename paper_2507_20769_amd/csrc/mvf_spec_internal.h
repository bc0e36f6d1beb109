// mvf_spec_internal.h -- host interface of the specialised-kernel generator.
#pragma once
#include <string>
#include <vector>

#include "mvf.h"
#include "mvf_internal.h"

namespace mvf {

// Tangent components per pass and generated size (instruction-passes: root
// program lengths times passes per root); MVF_ELIMIT above the size limit.
int spec_plan(const Compiled &P, const mvf_spec_options *opt, int *chunk, int64_t *units);

// Segment budget of the checkpointed adjoint (intervals; <= 0: one segment),
// and the record count above which a root is segmented (INT32_MAX: none).
int spec_ckpt_budget(const Compiled &P, const mvf_spec_options *opt, int waves);
int spec_ckpt_min_records(const Compiled &P, const mvf_spec_options *opt, int waves);
// The checkpoint plan of the adjoint at the library's choices (two waves per
// SIMD): segments over all roots, intervals stored and loaded per subdomain.
void spec_ckpt_plan_stats(const Compiled &P, int32_t *segments, int32_t *stored, int32_t *loaded);

// The generated device source (compiled with the embedded device headers):
// forward kernels (grad FWD), reverse-mode kernels (REV) or both (AUTO).
// ck_count receives the checkpoint intervals per lane of the adjoint, units
// the instruction-passes generated.
std::string spec_source(const Compiled &P, int chunk, int waves, int grad, int ckpt_budget, int min_records,
                        int *ck_count, int64_t *units);

// hiprtc compilation for `arch` (or the on-disk cache's copy).
int spec_compile(const std::string &src, const std::string &arch, bool use_cache, std::vector<char> &code,
                 bool *from_cache, double *seconds);

// dynamic LDS of the specialised single-box kernel; gl gradient components
// per lane in LDS (the adjoint kernel's launch: the tape's, else 0)
size_t spec_lds_bytes(int tab_total, int m, int gl = 0);
int spec_gl_count(const Compiled &P, int waves);

}  // namespace mvf
