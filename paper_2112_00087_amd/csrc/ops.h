// Host-side interface of the operator kernels and solvers.
#pragma once

#include "ctx.h"
#include "krylov.h"

// Device pointers of the real operator parts (SELL layout).
struct OpParts {
  const double* K = nullptr;
  const double* M = nullptr;
  const double* Meta = nullptr;   // NULL: no absorption field
  const int* bidx = nullptr;      // per stored entry: boundary slot or -1
  const z_t* Bb = nullptr;        // per boundary slot: sum_w beta_w B0_w
  const int* diag = nullptr;      // per row: stored position of the diagonal
  const uint8_t* emask = nullptr; // Dirichlet elimination per entry (NULL: none)
  double gls_h = 0.0;             // GLS element size (0: Galerkin mass coefficient)
};

// Mass coefficient m(k) of A = K - m(k) M + ...: k^2, or with the Galerkin
// least-squares stabilisation of Harari and Hughes (1992) for linear
// elements k^2 (1 - tau k^2), tau k^2 = 1 - 6 (1 - cos kh) / ((kh)^2 (2 +
// cos kh)), the value that makes the 1-D discrete dispersion exact.
inline double mass_coefficient(double k, double gls_h) {
  const double k2 = k * k;
  if (!(gls_h > 0.0) || k == 0.0) return k2;
  const double t = k * gls_h, c = std::cos(t);
  const double tau_k2 = 1.0 - 6.0 * (1.0 - c) / (t * t * (2.0 + c));
  return k2 * (1.0 - tau_k2);
}

inline OpParts op_parts(hz_ctx ctx) {
  OpParts P;
  P.K = ctx->d_K.as<double>();
  P.M = ctx->d_M.as<double>();
  P.Meta = ctx->have_eta ? ctx->d_Meta.as<double>() : nullptr;
  P.bidx = ctx->d_bidx.as<int>();
  P.Bb = ctx->d_Bb.as<z_t>();
  P.diag = ctx->d_diag.as<int>();
  P.emask = ctx->dirichlet ? ctx->d_emask.as<uint8_t>() : nullptr;
  P.gls_h = ctx->h.gls_h;
  return P;
}

// The current operator in complex form.
inline SellOp<double> op_A_complex(hz_ctx ctx) {
  SellOp<double> A;
  A.ptr = ctx->d_sptr.as<int>();
  A.col = ctx->d_scol.as<int>();
  A.val = ctx->d_A.as<z_t>();
  return A;
}
inline SellOp<float> op_A32_complex(hz_ctx ctx) {
  SellOp<float> A;
  A.ptr = ctx->d_sptr.as<int>();
  A.col = ctx->d_scol.as<int>();
  A.val = ctx->d_A32.as<c_t>();
  return A;
}
// The same operator in split form (valid when ctx->have_split / have_split32).
template <typename T>
inline SellOp<T> op_split(hz_ctx ctx) {
  SellOp<T> A;
  A.ptr = ctx->d_sptr.as<int>();
  A.col = ctx->d_scol.as<int>();
  A.dcol = ctx->split_dcol ? ctx->d_dcol.as<int16_t>() : nullptr;
  A.imeta = ctx->d_imeta.as<ImSlice>();
  A.icol = ctx->d_icol.as<int>();
  A.re = sizeof(T) == 8 ? static_cast<T*>(ctx->d_R.p) : static_cast<T*>(ctx->d_R32.p);
  A.iim = sizeof(T) == 8 ? static_cast<T*>(ctx->d_I.p) : static_cast<T*>(ctx->d_I32.p);
  return A;
}
// The same in stencil form (valid when ctx->have_stencil / have_stencil32).
template <typename T>
inline SellOp<T> op_stencil(hz_ctx ctx) {
  SellOp<T> A = op_split<T>(ctx);   // imaginary lists
  A.st = sizeof(T) == 8 ? static_cast<T*>(ctx->d_S.p) : static_cast<T*>(ctx->d_S32.p);
  A.nrows = ctx->sell.n_rows;
  A.soff = ctx->soff;
  return A;
}
// The operator the solvers use: the stencil form, else the split form, when formed.
inline SellOp<double> op_A(hz_ctx ctx) {
  return ctx->have_stencil ? op_stencil<double>(ctx) : ctx->have_split ? op_split<double>(ctx) : op_A_complex(ctx);
}
inline SellOp<float> op_A32(hz_ctx ctx) {
  return ctx->have_stencil32 ? op_stencil<float>(ctx)
                             : ctx->have_split32 ? op_split<float>(ctx) : op_A32_complex(ctx);
}

int op_set_frequency(hz_ctx ctx, const OpParts& P, double k, int scale, bool want32);
// Forms A(k) (optionally column-scaled by 1/diag) on an explicit sliced-ELL
// system; rows i >= n or with diag[i] < 0 are padding (d = 1).
int op_form(hipStream_t s, int64_t n, int64_t nrows, int64_t npad, const int* col, const OpParts& P, double k,
            int scale, z_t* A, c_t* A32, z_t* d, z_t* dinv, double* R = nullptr, float* R32 = nullptr);
// I[q] = Im A[ipos[q]] (0 where ipos[q] < 0), and its FP32 copy when I32 is
// given: the imaginary lists of a split-form operator.
int op_split_im(hipStream_t s, int64_t ni, const int* ipos, const z_t* A, double* I, float* I32);
template <typename T>
int op_spmv(hipStream_t s, int64_t nrows, int64_t nout, const SellOp<T>& A, const cx<T>* x, cx<T>* y);
int op_mul(hipStream_t s, int64_t n, const z_t* a, const z_t* b, z_t* c);
int op_fill(hipStream_t s, int64_t n, z_t* y, z_t v);
int op_copy(hipStream_t s, int64_t n, const z_t* x, z_t* y);
int op_load(hz_ctx ctx, const z_t* g, z_t* f);
int op_dotc(hz_ctx ctx, int64_t n, const z_t* a, const z_t* b, double* out_dev);
// Dirichlet load in the internal numbering (padded vectors of nrows):
// f_i = g_i on D rows, f_i = -sum_{j in D} A_ij g_j on the others, with the
// entries of A before the elimination (paper Sec. 3.2 Dirichlet source).
int op_lift(hz_ctx ctx, const z_t* g, z_t* f);
// The same two kernels with the caller's partial-sum buffer (2 reduce_grid(n)
// doubles) on the given stream.
int op_dotc_into(hipStream_t stream, int64_t n, const z_t* a, const z_t* b, double* part, double* out_dev);

// ---------------------------------------------------------------- solvers
// Per-segment controls and results of one Krylov run.
struct KrylovCtl {
  double tol = 1e-8;              // relative to ||f_seg||
  int max_matvec = 20000;
  int restart = 30;               // GMRES
  int ell = 4;                    // BiCGStab(l)
  // TFQMR: a quasi-residual bound that has not halved over this many
  // half-steps ends the solve (0: never).  Set for complex64 inner solves
  // of the refinement, whose bound can stall above the inner tolerance.
  int stall_halfsteps = 0;
};
struct KrylovOut {
  std::vector<int> iters, matvecs, status;
  std::vector<double> relres_est, fnorm;
};

// Solve A u = f on every segment (u: in x0 / out), vectors of the storage
// type T, reductions and Krylov scalars in FP64.
template <typename T>
int bicgstab_run(hz_ctx ctx, const SegHost& S, const SellOp<T>& A, const cx<T>* f, cx<T>* u,
                 const KrylovCtl& ctl, KrylovOut* out, const std::string& tag);
template <typename T>
int gmres_run(hz_ctx ctx, const SegHost& S, const SellOp<T>& A, const cx<T>* f, cx<T>* u,
              const KrylovCtl& ctl, KrylovOut* out, const std::string& tag);
template <typename T>
int bicgstabl_run(hz_ctx ctx, const SegHost& S, const SellOp<T>& A, const cx<T>* f, cx<T>* u,
                  const KrylovCtl& ctl, KrylovOut* out, const std::string& tag);
template <typename T>
int tfqmr_run(hz_ctx ctx, const SegHost& S, const SellOp<T>& A, const cx<T>* f, cx<T>* u,
              const KrylovCtl& ctl, KrylovOut* out, const std::string& tag);
// Dispatch on opts->method (HZ_GMRES, HZ_BICGSTAB, HZ_BICGSTABL or HZ_TFQMR).
template <typename T>
int krylov_run(hz_ctx ctx, int method, const SegHost& S, const SellOp<T>& A, const cx<T>* f, cx<T>* u,
               const KrylovCtl& ctl, KrylovOut* out, const std::string& tag) {
  if (method == HZ_BICGSTAB) return bicgstab_run<T>(ctx, S, A, f, u, ctl, out, tag);
  if (method == HZ_BICGSTABL) return bicgstabl_run<T>(ctx, S, A, f, u, ctl, out, tag);
  if (method == HZ_TFQMR) return tfqmr_run<T>(ctx, S, A, f, u, ctl, out, tag);
  return gmres_run<T>(ctx, S, A, f, u, ctl, out, tag);
}

// ||f_seg - A u_seg||^2 per segment (FP64), written to host vector rr.
int true_residual(hz_ctx ctx, const SegHost& S, const SellOp<double>& A, const z_t* f, const z_t* u,
                  z_t* r, std::vector<double>* rr);
template <typename T>
int seg_norm2_t(hz_ctx ctx, const SegHost& S, const cx<T>* x, std::vector<double>* out);

// Segment layout of the context's single system (one segment, padded rows).
int ctx_single_seg(hz_ctx ctx, SegHost** out);
int seg_upload(hz_ctx ctx, SegHost* S, const std::string& tag);
