// Internal interface between the plan executor (runtime.hip) and the server.
#pragma once

#include <hip/hip_runtime.h>

#include <string>

#include "../../include/cor_utv.h"

namespace cor {

struct Plan;
struct Prob;

cor_status fail(cor_status st, const std::string& msg);
cor_status hip_fail(hipError_t e, const char* what);

// Build a plan for `count` problems.  async: allocate, upload and clear on
// `astream` (stream-ordered; no device-wide synchronisation).  ext_mem: use
// these ext_bytes of device memory instead of allocating (COR_E_INVAL if the
// plan needs more); uploads and the clear are enqueued on `astream`.
cor_status plan_create(const cor_problem* probs, int32_t count, const cor_opts* opts, Plan** out,
                       hipStream_t astream, bool async, void* ext_mem = nullptr,
                       size_t ext_bytes = 0);
cor_status plan_run(Plan* P, hipStream_t s);
cor_status plan_info(Plan* P, cor_info* infos, hipStream_t s);
void plan_destroy(Plan* P, hipStream_t s);
size_t plan_bytes(const Plan* P);
const Prob& plan_desc(const Plan* P, int i);
int plan_count(const Plan* P);
int plan_report(const Plan* P);
// Whether a problem can take the fused power step (COR_OK, else COR_E_INVAL
// with the reason in cor_last_error()).
cor_status fused_check(const cor_problem& p, int ulv);
// Device workspace of one decomposition with the given options (NULL: defaults).
size_t workspace_bytes(int64_t m, int64_t n, int32_t l, int prec, const cor_opts* opts = nullptr);

}  // namespace cor
