// Batched radiosity solve state (one or more cavities, 1..16 right-hand sides).
#pragma once

#include "krylov.hpp"

namespace hm {

// Caller arrays of one slot for a permuted gather / scatter.
struct SlotIO {
  const double* in;   // caller array of the slot (original order)
  double* out;
  int64_t ld;         // leading dimension of the caller array
  const int32_t* perm;
  int64_t xoff;
  int64_t n;
};

struct SolveResult {
  int iters = 0, outer = 0, matvecs = 0;
  int64_t bytes = 0;
  bool converged = true;
  bool fx = false;              // the plain product F x of the final iterate is in H64
  std::vector<double> rel_res;  // per system (slot-major, then column)
};

struct TransientResult {
  int steps_done = 0, newton_total = 0, newton_max = 0, matvecs = 0;
  double max_rel_residual = 0.0;
  bool nonfinite = false;  // a Newton residual was not finite: the run stopped there
};

// Everything one batched solve needs, kept between calls on the same set of
// matrices: the composition of their products, the systems, the Krylov
// workspaces and the permuted vectors (combined row space N x W).
struct Batch {
  std::vector<const hm_matrix*> mats;
  int nrhs = 1, W = 1;
  int64_t N = 0;
  std::unique_ptr<Composition> C;
  SysSet S;
  Krylov K64, K32;
  bool k64 = false, k32 = false;
  DevBuf Tp, epsp, omeps64, omeps32, b64, b32, x64, x32, r64, H64, g, g_eps, d_flag;
  // refinement: per system, still above the tolerance; then per slot
  // (matrix), holds such a system (the next residual product runs on those
  // slots only)
  DevBuf res_mask;
  // Tables of the caller's per-slot buffers, one per role, in pinned host
  // memory and on the device: an upload needs no stream synchronisation; a
  // role's host table is rewritten only once its previous upload has
  // completed (the role's event, normally long past).
  enum IoRole { IO_EPS = 0, IO_T, IO_J, IO_Q, IO_SRC, IO_HIST, IO_ROLES };
  std::vector<SlotIO> ios;  // per slot: perm, n, xoff
  std::unique_ptr<PinnedLease> ios_lease;  // pinned, IO_ROLES tables
  SlotIO* ios_h = nullptr;
  SlotIO* ios_hd = nullptr; // their device view
  hipEvent_t io_ev[IO_ROLES] = {};
  DevBuf d_ios;             // IO_ROLES tables
  std::unique_ptr<Batch> gb;  // width-1 batch for g = F C^-1 eps
  bool g_ready = false;
  // whether this call's emissivities differ from those g was computed for:
  // compared on the device as soon as they are gathered, read back into
  // pinned memory, looked at when the flux needs g
  std::unique_ptr<PinnedLease> eps_lease;
  int* eps_flag_h = nullptr;
  void* eps_flag_hd = nullptr;
  hipEvent_t eps_ev = nullptr;
  bool eps_pending = false;
  void compare_eps(hipStream_t s);
  // open cavities (eq. (35)): amb = 1 - clamp(F 1, 0, 1) per permuted row,
  // and the ambient's T^4 of the current call (open = false: closed cavity)
  DevBuf amb;
  bool amb_ready = false, open = false;
  double tamb4 = 0.0;
  // the inputs T are radiation powers eta (any sign) instead of
  // temperatures: the right-hand side is sigma eps eta, the flux
  // eps (F J - sigma eta g) (the finite-element coupling's facet powers)
  bool power_in = false;

  Batch(const std::vector<const hm_matrix*>& mats, int nrhs, hipStream_t s);
  ~Batch();
  Batch(const Batch&) = delete;
  Batch& operator=(const Batch&) = delete;
  Krylov& krylov(int vb, int restart, hipStream_t s);
  void io(int role, const std::vector<const double*>& in, const std::vector<double*>& out, int64_t ld_in_default,
          const std::vector<int64_t>* lds, hipStream_t s);
  void gather(int role, double* dst, int ncol, int dst_cols, hipStream_t s);
  void scatter(int role, const double* src, int ncol, hipStream_t s);
  void ensure_g(const std::vector<const double*>& eps_user, hipStream_t s);
  // sets open / tamb4 from p and, for an open cavity, computes amb once
  void set_ambient(const hm_solve_params& p, hipStream_t s);
  void prepare_rhs(double sigma, const hm_solve_params& p, hipStream_t s);
  // report: with FP32 vectors, measure the final residual with FP64 vectors
  // (one more product; callers that check their own residual skip it)
  // keep_fx: with refinement, let the residual products leave F x in H64 too
  // (the flux then needs no product of its own)
  SolveResult solve_prepared(const hm_solve_params& p, hipStream_t s, bool warm = false, bool report = true,
                             bool keep_fx = false);
  // slot_active: NULL for every slot, else a device flag per slot
  void residual64(bool hi, hipStream_t s, bool keep_fx = false, const int* slot_active = nullptr);
  void flux(double sigma, hipStream_t s, bool have_fx = false);
  SolveResult solve(const std::vector<const double*>& eps, const std::vector<const double*>& T,
                    const std::vector<int64_t>& ldT, double sigma, const hm_solve_params& p,
                    const std::vector<double*>& J, const std::vector<int64_t>& ldJ, const std::vector<double*>& q,
                    const std::vector<int64_t>& ldq, hipStream_t s);
  TransientResult transient(const std::vector<const double*>& eps, double* T, int64_t ldT, const double* src,
                            int64_t ldS, double sigma, const hm_transient_params& tp, const hm_solve_params& sp,
                            double* history, hipStream_t s);
};

}  // namespace hm
