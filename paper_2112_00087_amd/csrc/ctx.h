// Context of one assembled mesh: host assembly products, device arrays,
// the current operator and cached solver workspaces.
#pragma once

#include <complex>
#include <map>
#include <memory>
#include <string>
#include <vector>

#include "common.h"
#include "krylov.h"

// Sliced ELL with 64-row slices (one wave per slice): slice s holds rows
// [64 s, 64 s + 64); its entries are stored column-major, entry k of lane l
// at ptr[s] + 64 k + l.  Short rows are padded with (col = own row, value 0);
// the lanes of the last slice beyond n_rows are padded with (col 0, value 0).
struct SellHost {
  int32_t n_rows = 0, n_slices = 0;
  int64_t n_pad = 0;                 // stored entries including padding
  std::vector<int32_t> ptr;          // [n_slices + 1]
  std::vector<int32_t> col;          // [n_pad]
  std::vector<int64_t> src;          // [n_pad] CSR position of the entry or -1
};

// Host-side assembly products (CSR with sorted columns).
struct HostAsm {
  int32_t n = 0, ne = 0, nb = 0;
  int32_t npe = 8, npf = 4;          // nodes per element / boundary face (8, 4: Q1; 4, 3: P1)
  int32_t ntags = 6;                 // boundary tags: 6 walls (+ 6 interface directions)
  std::vector<int64_t> rowptr;
  std::vector<int32_t> col;
  std::vector<double> K, M, Meta;    // per CSR entry (Meta empty when eta is NULL)
  std::vector<int64_t> diag;         // CSR position of (i,i)
  // boundary entries: CSR position and per-tag face mass, [nbe][ntags]
  std::vector<int64_t> bpos;
  std::vector<double> bmass;
  // source-patch mass restricted to the patch rows
  std::vector<int32_t> prow;
  std::vector<int32_t> pptr, pcol;
  std::vector<double> pval;
  // mesh copy (hex: npe nodes per element, bface: npf per face)
  std::vector<double> xyz;
  std::vector<int32_t> hex, bface, btag;
  std::vector<uint8_t> bsrc;
  // node -> elements adjacency (ascending element id)
  std::vector<int64_t> n2e_ptr;
  std::vector<int32_t> n2e;
  // Dirichlet source: 1 for the nodes of the source faces (empty: Neumann)
  std::vector<uint8_t> dir;
  double gls_h = 0.0;                // GLS element size (0: Galerkin)
};

// Validates and assembles a mesh.  With perm non-NULL the mesh's order and
// sigma fields are honoured: the assembly is then in the internal numbering
// and perm receives it (left empty for the mesh's own numbering).
int host_assemble(const hz_mesh* mesh, const double* eta, HostAsm* out, int ntags = 6,
                  std::vector<int32_t>* perm = nullptr);
// CSR pattern of the node graph of a mesh with npe nodes per element (row i:
// the sorted nodes of the elements around node i) and the node -> element
// adjacency.
int mesh_pattern(int64_t n, int64_t ne, int npe, const int32_t* hex, std::vector<int64_t>* n2e_ptr,
                 std::vector<int32_t>* n2e, std::vector<int64_t>* rowptr, std::vector<int32_t>* col);
// Internal node numbering for a pattern: position p holds node perm[p].
// order HZ_ORDER_RCM: reverse Cuthill-McKee; sigma > 0: rows sorted by
// length (longest first) within windows of sigma consecutive positions.
void node_order(int64_t n, const std::vector<int64_t>& rowptr, const std::vector<int32_t>& col, int order,
                int sigma, std::vector<int32_t>* perm);
int host_assemble_meta(HostAsm* a, const double* eta);
void build_sell(const HostAsm& a, int64_t nrows, SellHost* s);

// A device buffer that remembers its size.
struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  ~DevBuf() { if (p) (void)hipFree(p); }
  int ensure(size_t nbytes);     // grows (contents lost)
  template <typename T> T* as() const { return static_cast<T*>(p); }
};

struct hz_ctx_s {
  int device = 0;
  hipStream_t stream = nullptr;
  double c = 340.0, rho = 1.2;
  int32_t elems[3] = {0, 0, 0}, parts[3] = {0, 0, 0};
  HostAsm h;                         // assembled in the internal node numbering
  SellHost sell;
  // internal numbering: internal node p is the caller's node perm[p] (empty:
  // the caller's numbering); vectors cross the C ABI in the caller's order
  std::vector<int32_t> perm;
  DevBuf d_perm;
  int64_t dev_bytes = 0;

  // device pattern + real values in SELL layout
  DevBuf d_sptr, d_scol, d_K, d_M, d_Meta, d_bidx, d_diag;
  // boundary entries (SELL position, beta-weighted complex value)
  DevBuf d_bsell, d_Bb;
  DevBuf d_bmass;   // [nbe][6] per-wall masses (for gradients)
  // patch load CSR
  DevBuf d_prow, d_pptr, d_pcol, d_pval;
  // Dirichlet source: per stored entry 0 keep, 1 zero, 2 one (a D row's
  // diagonal); per internal row and per mesh node 1 for the nodes of D
  bool dirichlet = false;
  DevBuf d_emask, d_dirrow, d_dirmesh;
  // mesh on device (gradients)
  DevBuf d_xyz, d_hex, d_bface, d_btag;

  // current operator
  bool have_freq = false;
  double freq = 0.0, k = 0.0;
  int scaled = -1;                   // precond the operator values are scaled for
  DevBuf d_A, d_A32, d_d, d_dinv;    // A (maybe column-scaled), complex64 copy, diag, 1/diag
  bool have_A32 = false;

  // split form of the operator (real parts of every stored entry, imaginary
  // parts of the entries next to the absorbing walls); pattern built at
  // upload, values formed with A when there is no absorption field
  bool split_on = true;              // HZ_SPLIT=0 in the environment turns it off
  bool split_dcol = false;           // every |col - row| fits int16
  int64_t n_imag = 0;                // entries with a possibly nonzero imaginary part
  int64_t n_islots = 0;              // their interleaved slots (lists padded per slice)
  DevBuf d_dcol, d_imeta, d_icol, d_ipos;   // per slot: column, position in A (-1: padding)
  DevBuf d_R, d_R32, d_I, d_I32;
  bool have_split = false, have_split32 = false;   // values match the current A / A32

  // stencil form of the split values (structured boxes in their own node
  // numbering; HZ_STENCIL=0 in the environment turns it off): per slot the
  // sliced-ELL position it copies, or -1 for a missing neighbour
  bool stencil_ok = false;
  StencilOffsets soff = {};
  DevBuf d_ssrc, d_S, d_S32;
  bool have_stencil = false, have_stencil32 = false;

  std::vector<std::complex<double>> beta;   // [6]
  bool have_eta = false;
  int params_version = 0;            // bumped by hz_set_params

  // row-wise (CSR) copy of the real parts for the multi-vector product of
  // the frequency sweep, built on first use for a params_version
  int sweep_version = -1;
  std::shared_ptr<void> sweep_data;  // owned row-wise operator data of the sweep
  int dd_version = -1;
  std::shared_ptr<void> dd_data;     // owned subdomain systems of the Schwarz method
  std::vector<double> eta_field;     // per-element loss factors (empty: none)
  std::map<std::string, int> tuned;  // autotuned multi-vector product variants

  // scratch for solvers, keyed by name
  std::map<std::string, std::unique_ptr<DevBuf>> ws;
  std::unique_ptr<SegHost> single_seg;
  void* pinned = nullptr;            // small pinned host buffer for status reads
  size_t pinned_bytes = 0;

  DevBuf* buf(const std::string& name, size_t bytes, int* rc);
  ~hz_ctx_s();
};

int ctx_upload(hz_ctx ctx);
inline const int* ctx_perm(hz_ctx ctx) { return ctx->perm.empty() ? nullptr : ctx->d_perm.as<int>(); }
int ctx_upload_params(hz_ctx ctx);
int ctx_pinned(hz_ctx ctx, size_t bytes, void** out);
