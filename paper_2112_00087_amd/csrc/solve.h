// Solve drivers shared by the entry points.
#pragma once

#include "ops.h"

struct IrOut {
  int outer = 0;
  int64_t matvecs = 0, inner_matvecs = 0;
  int inner_status = HZ_OK;
  std::vector<double> relres, fnorm;
};

int ensure_operator(hz_ctx ctx, int precond, bool want32);
// Caller-ordered vector -> padded internal vector (optionally scaled per
// internal row), and back; both apply the context's node numbering.
int pad_in(hz_ctx ctx, int64_t n, int64_t nrows, const z_t* x, const z_t* scale, z_t* y);
int unpad_out(hz_ctx ctx, int64_t n, const z_t* u, const z_t* scale, z_t* p);
int ir_run(hz_ctx ctx, const SegHost& S, const SellOp<double>& A64, const SellOp<float>& A32,
           const z_t* f, z_t* u, const hz_solve_opts& o, IrOut* out, const std::string& tag);
int solve_single(hz_ctx ctx, const hz_solve_opts& o, const z_t* f, z_t* p, hz_solve_info* info);
int validate_opts(const hz_solve_opts* o);
