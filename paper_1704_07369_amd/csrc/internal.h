// Internal interfaces shared by the C-ABI translation units (not exported).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>

struct ec_batch;
struct ec_plan;

namespace efm {

// record an error message for ec_last_error() and return code
int set_error(int code, const std::string& msg);

// read-only views of a batch
const int64_t* batch_offsets_dev(const ec_batch* b);
int64_t batch_cells(const ec_batch* b);
int64_t batch_elems(const ec_batch* b);
int batch_groups(const ec_batch* b);
const ec_plan* batch_group_plan(const ec_batch* b, int g);
int64_t batch_group_count(const ec_batch* b, int g);
int plan_N(const ec_plan* p);
int plan_d(const ec_plan* p);
double plan_L(const ec_plan* p);
int plan_J(const ec_plan* p);
int plan_device(const ec_plan* p);
// the plan's device tables in FP64 (precision 0) or FP32; null if the plan
// keeps no copy in that precision
const void* plan_gamma(const ec_plan* p, int precision);

// x split that the fused schedule's defaults pick for launches of `cells`
// cells of N^3 (0: no fused schedule for N and precision)
int fused_split_for_cells(int N, int precision, int64_t cells);

// Q for the first n_active cells of group 0 only (the other cells untouched)
int collide_prefix(ec_batch* b, int64_t n_active, const double* f, double* Q, hipStream_t s);

}  // namespace efm
