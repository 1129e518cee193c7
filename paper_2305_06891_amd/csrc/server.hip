// Serving loop: radiosity solves of registered cavities, continuously
// batched.  A background host thread owns the solves; a second one
// assembles cavities that are not resident, on its own stream, while the
// admitted requests keep their rounds.  Requests are admitted while the
// resident H-matrices and the solve buffers fit the HBM budget; all admitted requests advance together, one refinement round at a
// time (FP64 residual with the most accurate stored factors, then an inner
// FP32 GMRES with the stored factors), sharing every H-matrix product and
// every Krylov kernel launch; requests that arrive meanwhile join at the
// next round, and converged requests leave with their radiosity and flux.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <deque>
#include <map>
#include <thread>

#include "convergence.hpp"
#include "dev_common.hpp"
#include "solve.hpp"

namespace hm {

hm_matrix* assemble(hm_ctx& ctx, const hm_tree& t, const hm_assembly_params& p);
int64_t matrix_bytes(const hm_matrix& M, bool hi);

namespace {

double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

template <class VT>
__global__ void k_srv_gather(const int32_t* __restrict__ perm, const double* __restrict__ in, int64_t ldi,
                             VT* __restrict__ out, int64_t ldo, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int j = blockIdx.y;
  if (i < n) out[i + j * ldo] = (VT)in[perm[i] + j * ldi];
}

__global__ void k_srv_scatter(const int32_t* __restrict__ perm, const double* __restrict__ in, int64_t ldi,
                              double* __restrict__ out, int64_t ldo, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int j = blockIdx.y;
  if (i < n) out[perm[i] + j * ldo] = in[i + j * ldi];
}

// b = sigma eps T^4 (permuted)
__global__ void k_srv_rhs(const double* __restrict__ eps, const double* __restrict__ T, double* __restrict__ b,
                          int64_t n, double sigma) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int j = blockIdx.y;
  if (i < n) {
    const double t = T[i + j * n];
    const double t2 = t * t;
    b[i + j * n] = sigma * eps[i] * (t2 * t2);
  }
}

__global__ void k_srv_flux(const double* __restrict__ eps, const double* __restrict__ T, const double* __restrict__ H,
                           const double* __restrict__ g, double* __restrict__ q, int64_t n, double sigma) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int j = blockIdx.y;
  if (i < n) {
    const double t = T[i + j * n];
    const double t2 = t * t;
    q[i + j * n] = eps[i] * (H[i + j * n] - sigma * (t2 * t2) * g[i]);
  }
}

template <class A, class B>
__global__ void k_srv_cast(const A* __restrict__ a, B* __restrict__ b, int64_t n) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n) b[k] = (B)a[k];
}

__global__ void k_srv_acc(const float* __restrict__ x, double* __restrict__ y, int64_t n) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n) y[k] += (double)x[k];
}

dim3 g2(int64_t n, int cols) { return dim3((unsigned)((n + 255) / 256), (unsigned)cols); }

}  // namespace

struct SrvCavity {
  uint64_t id = 0;
  std::unique_ptr<hm_tree> tree;
  std::vector<double> eps;
  hm_assembly_params ap{};
  hm_matrix* M = nullptr;
  DevBuf eps_d;          // original order
  DevBuf epsp, om64;     // permuted eps, 1 - eps
  DevBuf om32;
  DevBuf g;              // F C^-1 eps, permuted
  int64_t bytes = 0;     // device bytes while resident
  uint64_t last_use = 0;
  int refs = 0;
  bool building = false;  // queued for or in assembly on the assembler thread
  int waiting = 0;        // parked requests not yet admitted (the cavity is not evicted)
  int64_t reserved = 0;   // budget bytes held while building
  ~SrvCavity() { delete M; }
};

struct SrvReq {
  uint64_t ticket = 0, cid = 0;
  int nrhs = 0;
  int64_t n = 0;
  std::vector<double> T;          // host, original order, n x nrhs
  DevBuf Tp, b64, J64;            // device, permuted, n x nrhs
  std::vector<double> J, q;       // results (host)
  hm_status status = HM_OK;
  bool done = false;
  double t_submit = 0, t_done = 0;
  int rounds = 0, inner = 0, matvecs = 0;
  int64_t bytes = 0;
  double rel_res = 0;
  bool waited = false;  // parked while its cavity was assembled
};

}  // namespace hm

struct hm_server {
  hm_server_params p{};
  int device = 0;
  hipStream_t stream = nullptr;
  std::mutex mu;
  std::condition_variable cv;
  std::map<uint64_t, std::unique_ptr<hm::SrvCavity>> cav;
  std::map<uint64_t, std::unique_ptr<hm::SrvReq>> req;
  std::deque<uint64_t> queue;
  std::vector<uint64_t> active;
  std::vector<uint64_t> parked;       // requests waiting for their cavity's assembly
  std::vector<uint64_t> ready;        // parked requests whose cavity is built (the worker
                                      // moves them to the queue front: only it pops the queue)
  std::deque<uint64_t> build_queue;   // cavities to assemble, in order
  std::condition_variable acv;
  uint64_t next_ticket = 1, clock = 0;
  bool stop = false;
  hm_server_stats st{};
  std::thread worker, assembler;
  hm_ctx ctx;   // the worker's own context (device + private stream)
  hm_ctx actx;  // the assembler's (device + its own stream)
  // storage types shared by every cavity (set by the first registration):
  // a round composes all active cavities into one product
  bool have_types = false;
  hm_dtype lr_type = HM_F32, dense_type = HM_F32;
  int32_t keep_copy = 0;
  enum Admit { ADMITTED, PARKED, WAIT, REJECTED };
  void run();
  void build_loop();
  void round(std::vector<hm::SrvReq*>& act);
  Admit admit_one(hm::SrvReq& r);
  void park_locked(hm::SrvReq& r);
  int64_t resident() const;
  int64_t active_need_locked(const hm::SrvReq* extra, int64_t extra_ktot) const;
};

using namespace hm;

int64_t hm_server::resident() const {
  int64_t b = 0;
  for (auto& kv : cav) {
    if (kv.second->M) b += kv.second->bytes;
    else if (kv.second->building) b += kv.second->reserved;
  }
  return b;
}

namespace hm {
namespace {
// Device bytes of one request's own vectors (temperatures, right-hand side,
// radiosity; FP64, permuted).
int64_t req_bytes(int64_t n, int nrhs) { return 3 * 8 * n * (int64_t)nrhs; }

// Device bytes of one round over requests with `rows` rows in total, padded
// width W and sum_ktot rank columns: the round's FP64 and FP32 vectors (b, x,
// r, F x; b, x), the FP64 Krylov workspace of the residual norms (restart 1)
// and the FP32 one of the inner GMRES (restart + 1 basis blocks, w, r), the
// product's rank-column intermediates and row-major inputs, the flux
// buffers of finishing requests and the per-row emissivity factors.
int64_t round_bytes(int64_t rows, int W, int restart, int64_t sum_ktot, int64_t nsys) {
  const int64_t blk = rows * W;
  int64_t b = blk * (4 * 8 + 2 * 4);           // b64 x64 r64 H, b32 x32
  b += blk * 8 * 4;                             // K8: 2 basis blocks, w, r
  b += blk * 4 * (int64_t)(restart + 3);        // K4: restart + 1 basis blocks, w, r
  b += blk * 8 * 5;                             // flux and result buffers of finishing requests
  b += sum_ktot * W * 8;                        // t
  if (W == 16) b += blk * 8;                    // row-major inputs of 16-column products
  b += rows * 12;                               // 1 - eps, FP64 and FP32
  b += nsys * (80 << 10);                       // Hessenberg data and rotations of each system
  return b + (64 << 10);                        // descriptors and reduction partials
}
}  // namespace
}  // namespace hm

// Bytes the active requests need (their own vectors and one shared round),
// with `extra` added (may be NULL) whose cavity has extra_ktot rank columns.
// Caller holds the lock.
int64_t hm_server::active_need_locked(const SrvReq* extra, int64_t extra_ktot) const {
  int64_t rows = 0, kt = 0, own = 0, nsys = 0;
  int maxr = 1;
  auto add = [&](const SrvReq& r, int64_t ktot) {
    rows += r.n;
    kt += ktot;
    own += req_bytes(r.n, r.nrhs);
    nsys += r.nrhs;
    maxr = std::max(maxr, r.nrhs);
  };
  for (uint64_t tk : active) {
    auto it = req.find(tk);
    if (it == req.end()) continue;
    const SrvReq& r = *it->second;
    auto ci = cav.find(r.cid);
    add(r, ci != cav.end() && ci->second->M ? ci->second->M->Ktot : 4 * r.n);
  }
  if (extra) add(*extra, extra_ktot);
  if (rows == 0) return 0;
  return own + round_bytes(rows, pad_width(maxr), p.solve.restart, kt, nsys);
}

// Moves the request at the queue front to the parked list (caller holds the
// lock).  Parking happens in the same critical section that sees its cavity
// queued for or in assembly: the assembler hands back the parked requests of
// a cavity when its build ends, so a request parked after that would wait
// forever.
void hm_server::park_locked(SrvReq& r) {
  if (!queue.empty() && queue.front() == r.ticket) queue.pop_front();
  if (!r.waited) cav.at(r.cid)->waiting++;
  r.waited = true;
  parked.push_back(r.ticket);
}

// Admit a request whose cavity is resident (allocate its vectors); for a
// cavity that is not, make room in the budget (evicting idle cavities, least
// recently used first) and hand it to the assembler thread, parking the
// request until the cavity is built, so that the requests already running
// keep their rounds meanwhile.  Called without the lock held, for the
// request at the queue front; device state of resident cavities is touched
// only by the worker thread.
hm_server::Admit hm_server::admit_one(SrvReq& r) {
  SrvCavity* c;
  bool res;
  int64_t built_bytes;
  {
    std::lock_guard<std::mutex> lk(mu);
    c = cav.at(r.cid).get();
    if (c->building) {
      park_locked(r);
      return PARKED;
    }
    res = c->M != nullptr;
    built_bytes = c->bytes;
  }
  // the cavity (when it is not resident: its size when it was last built,
  // else an estimate), this request's vectors and the round it joins must
  // fit beside what is resident or being built
  const int64_t cav_bytes = built_bytes > 0 ? built_bytes : r.n * 2500 * 4;
  const int64_t est = res ? 0 : cav_bytes;
  const int64_t ktot = res ? c->M->Ktot : 4 * r.n;
  // a request that cannot fit even alone fails (the cavity's size is known
  // once it has been built; before that only the request's own bytes count)
  const int64_t alone = (built_bytes > 0 ? built_bytes : 0) + req_bytes(r.n, r.nrhs) +
                        round_bytes(r.n, pad_width(r.nrhs), p.solve.restart, ktot, r.nrhs);
  if (alone > p.hbm_budget_bytes) return REJECTED;
  auto over_locked = [&] {
    std::lock_guard<std::mutex> lk(mu);
    return resident() + est + active_need_locked(&r, ktot) > p.hbm_budget_bytes;
  };
  {
    // evict idle cavities (least recently used first) until it fits
    for (;;) {
      if (!over_locked()) break;
      SrvCavity* lru = nullptr;
      {
        std::lock_guard<std::mutex> lk(mu);
        for (auto& kv : cav)
          if (kv.second.get() != c && kv.second->M && kv.second->refs == 0 && kv.second->waiting == 0 &&
              (!lru || kv.second->last_use < lru->last_use))
            lru = kv.second.get();
      }
      if (!lru) break;
      HM_HIP(hipStreamSynchronize(stream));
      hm_matrix* dead;
      {
        std::lock_guard<std::mutex> lk(mu);
        dead = lru->M;
        lru->M = nullptr;
        st.evictions++;
      }
      delete dead;
      lru->epsp.release();
      lru->om64.release();
      lru->om32.release();
      lru->g.release();
    }
  }
  {
    std::lock_guard<std::mutex> lk(mu);
    if (resident() + est + active_need_locked(&r, ktot) > p.hbm_budget_bytes) {
      // running requests or builds hold the budget: wait for them (with
      // nothing running or building, every idle cavity has been evicted and
      // the request fits alone, so this cannot wait forever)
      const bool busy = !active.empty() || !build_queue.empty();
      if (busy) return WAIT;
    }
    if (!res) {
      c->building = true;
      c->reserved = est;
      build_queue.push_back(c->id);
      park_locked(r);
      acv.notify_all();
      return PARKED;
    }
  }
  {
    std::lock_guard<std::mutex> lk(mu);
    if (!r.waited) st.cache_hits++;
    else c->waiting--;
    c->refs++;
    c->last_use = ++clock;
  }
  // request vectors (permuted)
  const int64_t n = r.n;
  DevBuf Th(n * r.nrhs * 8);
  HM_HIP(hipMemcpyAsync(Th.get(), r.T.data(), n * r.nrhs * 8, hipMemcpyHostToDevice, stream));
  r.Tp.alloc(n * r.nrhs * 8);
  r.b64.alloc(n * r.nrhs * 8);
  r.J64.alloc(n * r.nrhs * 8);
  hipLaunchKernelGGL(k_srv_gather<double>, g2(n, r.nrhs), dim3(256), 0, stream, c->M->d_perm.get<int32_t>(),
                     Th.get<double>(), n, r.Tp.get<double>(), n, n);
  hipLaunchKernelGGL(k_srv_rhs, g2(n, r.nrhs), dim3(256), 0, stream, c->epsp.get<double>(), r.Tp.get<double>(),
                     r.b64.get<double>(), n, p.sigma);
  HM_HIP(hipMemsetAsync(r.J64.get(), 0, n * r.nrhs * 8, stream));
  HM_HIP(hipStreamSynchronize(stream));
  return ADMITTED;
}

// The assembler thread: H-matrix, permuted emissivities and g = F C^-1 eps
// (eq. (12)) of each queued cavity, on its own stream; then the requests
// parked for the cavity are handed back (the worker puts them at the front
// of the queue in their order).
void hm_server::build_loop() {
  (void)hipSetDevice(device);
  set_current_stream(actx.stream);
  for (;;) {
    SrvCavity* c;
    {
      std::unique_lock<std::mutex> lk(mu);
      acv.wait(lk, [&] { return stop || !build_queue.empty(); });
      if (stop) return;
      c = cav.at(build_queue.front()).get();
    }
    hipStream_t as = actx.stream;
    hm_matrix* M = nullptr;
    bool ok = true;
    try {
      M = assemble(actx, *c->tree, c->ap);
      M->id = 0x8000000000000000ull | c->id;
      const int64_t n = M->n;
      c->eps_d.alloc(n * 8);
      HM_HIP(hipMemcpyAsync(c->eps_d.get(), c->eps.data(), n * 8, hipMemcpyHostToDevice, as));
      c->epsp.alloc(n * 8);
      hipLaunchKernelGGL(k_srv_gather<double>, g2(n, 1), dim3(256), 0, as, M->d_perm.get<int32_t>(),
                         c->eps_d.get<double>(), n, c->epsp.get<double>(), n, n);
      std::vector<double> om(n);
      for (int64_t i = 0; i < n; ++i) om[i] = 1.0 - c->eps[M->perm[i]];
      std::vector<float> om32(om.begin(), om.end());
      upload(c->om64, om, as);
      upload(c->om32, om32, as);
      {
        Batch B({M}, 1, as);
        B.io(Batch::IO_EPS, {c->eps_d.get<double>()}, {}, 0, nullptr, as);
        B.gather(Batch::IO_EPS, B.epsp.get<double>(), 1, 1, as);
        B.ensure_g({c->eps_d.get<double>()}, as);
        c->g.alloc(n * 8);
        HM_HIP(hipMemcpyAsync(c->g.get(), B.g.get(), n * 8, hipMemcpyDeviceToDevice, as));
        HM_HIP(hipStreamSynchronize(as));
      }
    } catch (const std::exception& e) {
      (void)hipGetLastError();
      delete M;
      M = nullptr;
      ok = false;
      actx.last_error = e.what();
    }
    std::lock_guard<std::mutex> lk(mu);
    build_queue.pop_front();
    c->building = false;
    c->reserved = 0;
    if (ok) {
      c->M = M;
      c->bytes = M->bytes_device() + M->n * 8 * 4;
      st.assemblies++;
    }
    // the cavity's parked requests: back to the queue front, or failed
    std::vector<uint64_t> back, keep;
    for (uint64_t tk : parked) {
      SrvReq& r = *req.at(tk);
      if (r.cid != c->id) {
        keep.push_back(tk);
      } else if (ok) {
        back.push_back(tk);
      } else {
        c->waiting--;
        r.status = HM_EDEVICE;
        r.t_done = now_s();
        r.done = true;
      }
    }
    parked.swap(keep);
    ready.insert(ready.end(), back.begin(), back.end());
    cv.notify_all();
  }
}

// One refinement round for every active request.
void hm_server::round(std::vector<SrvReq*>& act) {
  hipStream_t s = stream;
  std::vector<const hm_matrix*> mats;
  std::vector<SrvCavity*> cs;
  int maxr = 1;
  {
    std::lock_guard<std::mutex> lk(mu);
    for (auto* r : act) {
      SrvCavity* c = cav.at(r->cid).get();
      cs.push_back(c);
      mats.push_back(c->M);
      maxr = std::max(maxr, r->nrhs);
    }
  }
  const int W = pad_width(maxr);
  auto C = make_composition(mats, W, 8, s);
  const int64_t N = C->N;
  std::vector<std::vector<int>> cols(act.size());
  for (size_t q = 0; q < act.size(); ++q)
    for (int j = 0; j < act[q]->nrhs; ++j) cols[q].push_back(j);
  SysSet S;
  S.build(*C, cols, s);
  const size_t blk = (size_t)N * W;
  DevBuf b64(blk * 8), x64(blk * 8), r64(blk * 8), om64(N * 8), om32(N * 4), b32(blk * 4), x32(blk * 4);
  HM_HIP(hipMemsetAsync(b64.get(), 0, blk * 8, s));
  HM_HIP(hipMemsetAsync(x64.get(), 0, blk * 8, s));
  for (size_t q = 0; q < act.size(); ++q) {
    const int64_t off = C->xoff[q], n = act[q]->n;
    HM_HIP(hipMemcpy2DAsync(b64.get<double>() + off, N * 8, act[q]->b64.get(), n * 8, n * 8, act[q]->nrhs,
                            hipMemcpyDeviceToDevice, s));
    HM_HIP(hipMemcpy2DAsync(x64.get<double>() + off, N * 8, act[q]->J64.get(), n * 8, n * 8, act[q]->nrhs,
                            hipMemcpyDeviceToDevice, s));
    HM_HIP(hipMemcpyAsync(om64.get<double>() + off, cs[q]->om64.get(), n * 8, hipMemcpyDeviceToDevice, s));
    HM_HIP(hipMemcpyAsync(om32.get<float>() + off, cs[q]->om32.get(), n * 4, hipMemcpyDeviceToDevice, s));
  }
  // FP64 residual r = b - C J with the most accurate stored factors; the
  // product also leaves H = F J, the flux of the requests that finish now
  DevBuf H(blk * 8);
  Epilogue ep;
  ep.rowscale = om64.get();
  ep.a_acc = 1.0;
  ep.a_x = -1.0;
  ep.a_z = 1.0;
  ep.z = b64.get();
  ep.ldz = N;
  ep.acc_out = H.get();
  ep.ld_acc = N;
  launch_matvec(*C, W, 8, true, x64.get(), N, r64.get(), N, ep, nullptr, s);
  Krylov K8;
  K8.init(*C, S, 8, 1, s);
  std::vector<double> rn, bn;
  block_norms(K8, r64.get(), rn, s);
  block_norms(K8, b64.get(), bn, s);
  // per request: converged?
  std::vector<int> fin(act.size(), 1);
  std::vector<double> worst(act.size(), 0.0);
  for (int k = 0; k < S.size(); ++k) {
    const int q = S.sys[k].slot;
    worst[q] = max_keep_nan(worst[q], rel_residual(rn[k], bn[k]));
    if (!residual_met(rn[k], bn[k], p.solve.rtol)) fin[q] = 0;
  }
  for (size_t q = 0; q < act.size(); ++q) {
    act[q]->matvecs++;
    act[q]->bytes += matrix_bytes(*mats[q], true);
    act[q]->rel_res = worst[q];
    // give up after 40 rounds, or at once on a residual that is not finite:
    // reported as not converged
    if (!fin[q] && (act[q]->rounds >= 40 || std::isnan(worst[q]))) fin[q] = 1;
  }
  // finishing requests: flux and results
  bool any_fin = false;
  for (size_t q = 0; q < act.size(); ++q) any_fin |= fin[q] != 0;
  if (any_fin) {
    for (size_t q = 0; q < act.size(); ++q) {
      if (!fin[q]) continue;
      SrvReq& r = *act[q];
      const int64_t n = r.n, off = C->xoff[q];
      DevBuf Hq(n * r.nrhs * 8), Jq(n * r.nrhs * 8), qq(n * r.nrhs * 8), Jo(n * r.nrhs * 8), qo(n * r.nrhs * 8);
      HM_HIP(hipMemcpy2DAsync(Hq.get(), n * 8, H.get<double>() + off, N * 8, n * 8, r.nrhs, hipMemcpyDeviceToDevice, s));
      HM_HIP(hipMemcpy2DAsync(Jq.get(), n * 8, x64.get<double>() + off, N * 8, n * 8, r.nrhs, hipMemcpyDeviceToDevice, s));
      hipLaunchKernelGGL(k_srv_flux, g2(n, r.nrhs), dim3(256), 0, s, cs[q]->epsp.get<double>(), r.Tp.get<double>(),
                         Hq.get<double>(), cs[q]->g.get<double>(), qq.get<double>(), n, p.sigma);
      hipLaunchKernelGGL(k_srv_scatter, g2(n, r.nrhs), dim3(256), 0, s, mats[q]->d_perm.get<int32_t>(),
                         Jq.get<double>(), n, Jo.get<double>(), n, n);
      hipLaunchKernelGGL(k_srv_scatter, g2(n, r.nrhs), dim3(256), 0, s, mats[q]->d_perm.get<int32_t>(),
                         qq.get<double>(), n, qo.get<double>(), n, n);
      r.J.resize(n * r.nrhs);
      r.q.resize(n * r.nrhs);
      HM_HIP(hipMemcpyAsync(r.J.data(), Jo.get(), n * r.nrhs * 8, hipMemcpyDeviceToHost, s));
      HM_HIP(hipMemcpyAsync(r.q.data(), qo.get(), n * r.nrhs * 8, hipMemcpyDeviceToHost, s));
      HM_HIP(hipStreamSynchronize(s));
    }
  }
  // continuing requests: inner FP32 GMRES with the stored factors on C d = r.
  // The Krylov workspace lives until the round's closing synchronisation:
  // GMRES returns with its last update still queued, and the allocator hands
  // freed blocks to the assembler thread, whose stream does not wait for
  // this one.
  Krylov K4;
  bool any_cont = false;
  for (size_t q = 0; q < act.size(); ++q) any_cont |= !fin[q];
  if (any_cont) {
    hipLaunchKernelGGL((k_srv_cast<double, float>), dim3((unsigned)((blk + 255) / 256)), dim3(256), 0, s,
                       r64.get<double>(), b32.get<float>(), (int64_t)blk);
    for (int k = 0; k < S.size(); ++k) {
      const int q = S.sys[k].slot;
      if (fin[q] || residual_met(rn[k], bn[k], p.solve.rtol)) {
        const SysDev& sd = S.sys[k];
        HM_HIP(hipMemsetAsync(b32.get<float>() + sd.col * N + sd.row0, 0, (size_t)sd.n * 4, s));
      }
    }
    // correction from zero, stopped on the GMRES residual estimate (the
    // next round's FP64 residual checks it)
    HM_HIP(hipMemsetAsync(x32.get(), 0, blk * 4, s));
    K4.init(*C, S, 4, p.solve.restart, s);
    const double inner = p.solve.mixed_precision ? p.solve.ir_inner_rtol : std::min(p.solve.ir_inner_rtol, 1e-5);
    // one Gram-Schmidt pass per step at the loose tolerance of mixed rounds
    GmresStats gs = gmres(K4, false, om32.get(), b32.get(), x32.get(), inner, p.solve.max_iter, s, false,
                          GM_X0_ZERO | GM_TRUST_ESTIMATE | (p.solve.mixed_precision ? GM_CGS1 : 0u));
    hipLaunchKernelGGL(k_srv_acc, dim3((unsigned)((blk + 255) / 256)), dim3(256), 0, s, x32.get<float>(),
                       x64.get<double>(), (int64_t)blk);
    for (size_t q = 0; q < act.size(); ++q) {
      if (fin[q]) continue;
      SrvReq& r = *act[q];
      HM_HIP(hipMemcpy2DAsync(r.J64.get(), r.n * 8, x64.get<double>() + C->xoff[q], N * 8, r.n * 8, r.nrhs,
                              hipMemcpyDeviceToDevice, s));
      r.inner += gs.iters;
      r.matvecs += gs.matvecs;
      r.bytes += gs.bytes / (int64_t)act.size();
    }
  }
  HM_HIP(hipStreamSynchronize(s));
  // retire
  const double t = now_s();
  std::lock_guard<std::mutex> lk(mu);
  st.rounds++;
  for (size_t q = 0; q < act.size(); ++q) {
    SrvReq& r = *act[q];
    r.rounds++;
    if (!fin[q]) continue;
    r.Tp.release();
    r.b64.release();
    r.J64.release();
    cs[q]->refs--;
    st.completed++;
    // leave the active list in the same critical section that publishes the
    // result: once done is set the client may poll and erase the request
    active.erase(std::find(active.begin(), active.end(), r.ticket));
    r.done = true;
    r.t_done = t;
    r.status = rel_met(worst[q], p.solve.rtol) ? HM_OK : HM_ENOTCONV;
  }
}

void hm_server::run() {
  (void)hipSetDevice(device);
  set_current_stream(stream);
  for (;;) {
    std::vector<uint64_t> pending;
    {
      std::unique_lock<std::mutex> lk(mu);
      cv.wait(lk, [&] { return stop || !queue.empty() || !active.empty() || !ready.empty(); });
      if (stop && active.empty()) return;
    }
    const double t0 = now_s();
    bool no_room = false;  // the queue front waits for budget held by a build or by running requests
    try {
      // admission: FIFO while slots are free and the budget allows
      for (;;) {
        uint64_t tk = 0;
        {
          std::lock_guard<std::mutex> lk(mu);
          // requests whose cavity the assembler has built go first, in order
          queue.insert(queue.begin(), ready.begin(), ready.end());
          ready.clear();
          if (stop || queue.empty() || (int)active.size() >= p.max_active) break;
          tk = queue.front();
        }
        SrvReq* r;
        {
          std::lock_guard<std::mutex> lk(mu);
          r = req.at(tk).get();
        }
        Admit a = WAIT;
        try {
          a = admit_one(*r);
        } catch (const std::exception& e) {
          // this request cannot be admitted (assembly or allocation failed):
          // fail it alone and keep serving the others
          (void)hipGetLastError();
          const Error* he = dynamic_cast<const Error*>(&e);
          std::lock_guard<std::mutex> lk(mu);
          if (!queue.empty() && queue.front() == tk) queue.pop_front();
          if (r->waited) cav.at(r->cid)->waiting--;
          r->status = he ? he->code : HM_EDEVICE;
          r->t_done = now_s();
          r->done = true;
          ctx.last_error = e.what();
          continue;
        }
        std::lock_guard<std::mutex> lk(mu);
        if (a == REJECTED) {
          // needs more device memory than the whole budget: fail it alone
          if (!queue.empty() && queue.front() == tk) queue.pop_front();
          if (r->waited) cav.at(r->cid)->waiting--;
          r->status = HM_ENOMEM;
          r->t_done = now_s();
          r->done = true;
          st.rejected++;
          ctx.last_error = "request needs more device memory than the server's budget";
          continue;
        }
        if (a == WAIT) {
          no_room = true;
          break;
        }
        if (a == PARKED) continue;  // admit_one has moved it to the parked list
        if (queue.empty() || queue.front() != tk) break;  // the queue was cleared (shutdown)
        queue.pop_front();
        active.push_back(tk);
      }
      std::vector<SrvReq*> act;
      {
        std::lock_guard<std::mutex> lk(mu);
        for (uint64_t tk : active) act.push_back(req.at(tk).get());
      }
      if (!act.empty()) round(act);  // retires finished requests from active
      std::unique_lock<std::mutex> lk(mu);
      st.busy_seconds += now_s() - t0;
      st.resident_bytes = resident();
      // nothing running and the queue front waits for a build to release
      // budget: sleep until the assembler reports (bounded, no busy loop)
      if (no_room && act.empty())
        cv.wait_for(lk, std::chrono::milliseconds(2),
                    [&] { return stop || !ready.empty() || build_queue.empty(); });
    } catch (const std::exception& e) {
      // fail every active request with the error; keep serving
      (void)hipGetLastError();
      const Error* he = dynamic_cast<const Error*>(&e);
      std::lock_guard<std::mutex> lk(mu);
      for (uint64_t tk : active) {
        auto rit = req.find(tk);
        if (rit == req.end()) continue;
        SrvReq& r = *rit->second;
        auto it = cav.find(r.cid);
        if (it != cav.end() && it->second->refs > 0) it->second->refs--;
        r.status = he ? he->code : HM_EDEVICE;
        r.t_done = now_s();
        r.done = true;
      }
      active.clear();
      ctx.last_error = e.what();
    }
    cv.notify_all();
  }
}

extern "C" {

hm_status hm_server_create(hm_ctx* ctx, const hm_server_params* p, hm_server** out) {
  if (!ctx || !p || !out) {
    set_tl_error("hm_server_create: NULL argument");
    return HM_EINVAL;
  }
  try {
    HM_REQUIRE(p->hbm_budget_bytes > 0 && p->max_active >= 1, "hm_server_create: bad budget or max_active");
    HM_REQUIRE(p->max_rhs_per_slot >= 1 && p->max_rhs_per_slot <= 16, "hm_server_create: max_rhs_per_slot in 1..16");
    HM_REQUIRE(p->sigma > 0.0, "hm_server_create: sigma must be > 0");
    HM_REQUIRE(p->solve.open_cavity == 0, "hm_server_create: open cavities are not served (closed cavities only)");
    HM_REQUIRE(p->solve.rtol > 0 && p->solve.rtol < 1 && p->solve.restart >= 1 && p->solve.restart <= MAXM &&
                   p->solve.max_iter >= 1 && p->solve.ir_inner_rtol > 0 && p->solve.ir_inner_rtol < 1,
               "hm_server_create: bad solve parameters");
    auto s = std::make_unique<hm_server>();
    s->p = *p;
    s->device = ctx->device;
    HM_HIP(hipSetDevice(ctx->device));
    HM_HIP(hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking));
    s->ctx.device = ctx->device;
    s->ctx.stream = s->stream;
    s->actx.device = ctx->device;
    HM_HIP(hipStreamCreateWithFlags(&s->actx.stream, hipStreamNonBlocking));
    hm_server* raw = s.get();
    s->worker = std::thread([raw] { raw->run(); });
    s->assembler = std::thread([raw] { raw->build_loop(); });
    *out = s.release();
    return HM_OK;
  } catch (const Error& e) {
    ctx->last_error = e.what();
    set_tl_error(e.what());
    return e.code;
  }
}

hm_status hm_server_register_cavity(hm_server* s, uint64_t cid, const hm_tree* tree, const double* eps_host,
                                    const hm_assembly_params* ap) {
  if (!s || !tree || !eps_host || !ap) {
    set_tl_error("hm_server_register_cavity: NULL argument");
    return HM_EINVAL;
  }
  try {
    for (int64_t i = 0; i < tree->n; ++i)
      HM_REQUIRE(eps_host[i] > 0.0 && eps_host[i] <= 1.0, "hm_server_register_cavity: eps must be in (0, 1]");
    HM_REQUIRE(ap->aca_tol > 0 && ap->aca_tol < 1 && ap->k_max >= 1, "hm_server_register_cavity: bad assembly parameters");
    HM_REQUIRE(ap->dense_dtype != HM_BF16 || (ap->lowrank_dtype == HM_BF16 && ap->keep_f32_copy),
               "hm_server_register_cavity: a BF16 near field needs BF16 factors and keep_f32_copy");
    HM_REQUIRE(ap->lowrank_dtype != HM_BF16 || ap->keep_f32_copy,
               "hm_server_register_cavity: BF16 factors need keep_f32_copy (the FP64 residual reads the FP32 copies)");
    HM_REQUIRE(!(ap->dense_dtype == HM_F64 && ap->lowrank_dtype == HM_BF16),
               "hm_server_register_cavity: BF16 factors need an FP32 or BF16 near field");
    auto c = std::make_unique<SrvCavity>();
    c->id = cid;
    c->tree = std::make_unique<hm_tree>(*tree);
    c->eps.assign(eps_host, eps_host + tree->n);
    c->ap = *ap;
    c->ap.closed_row_scale = 0;
    std::lock_guard<std::mutex> lk(s->mu);
    HM_REQUIRE(s->cav.find(cid) == s->cav.end(), "hm_server_register_cavity: id already registered");
    const int32_t keep = ap->lowrank_dtype == HM_BF16 ? 1 : 0;
    if (s->have_types)
      HM_REQUIRE(ap->lowrank_dtype == s->lr_type && ap->dense_dtype == s->dense_type && keep == s->keep_copy,
                 "hm_server_register_cavity: every cavity of a server must use the storage types of the first "
                 "registered one (lowrank_dtype, dense_dtype, keep_f32_copy)");
    s->have_types = true;
    s->lr_type = ap->lowrank_dtype;
    s->dense_type = ap->dense_dtype;
    s->keep_copy = keep;
    s->cav[cid] = std::move(c);
    return HM_OK;
  } catch (const Error& e) {
    set_tl_error(e.what());
    return e.code;
  }
}

hm_status hm_submit(hm_server* s, uint64_t cid, int32_t nrhs, const double* T_host, uint64_t* ticket) {
  if (!s || !T_host || !ticket) {
    set_tl_error("hm_submit: NULL argument");
    return HM_EINVAL;
  }
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->cav.find(cid);
  if (it == s->cav.end()) {
    set_tl_error("hm_submit: unknown cavity id");
    return HM_ENOTFOUND;
  }
  if (nrhs < 1 || nrhs > s->p.max_rhs_per_slot) {
    set_tl_error("hm_submit: nrhs out of range");
    s->st.rejected++;
    return HM_EINVAL;
  }
  const int64_t n = it->second->tree->n;
  for (int64_t k = 0; k < n * nrhs; ++k)
    if (!(T_host[k] > 0.0) || !std::isfinite(T_host[k])) {
      set_tl_error("hm_submit: temperatures must be positive and finite");
      s->st.rejected++;
      return HM_EINVAL;
    }
  auto r = std::make_unique<SrvReq>();
  r->ticket = s->next_ticket++;
  r->cid = cid;
  r->nrhs = nrhs;
  r->n = n;
  r->T.assign(T_host, T_host + n * nrhs);
  r->t_submit = now_s();
  *ticket = r->ticket;
  s->queue.push_back(r->ticket);
  s->req[r->ticket] = std::move(r);
  s->st.submitted++;
  s->cv.notify_all();
  return HM_OK;
}

hm_status hm_poll(hm_server* s, uint64_t ticket, int32_t* done, double* J_host, double* q_host, hm_solve_info* info,
                  double* latency) {
  if (!s || !done) {
    set_tl_error("hm_poll: NULL argument");
    return HM_EINVAL;
  }
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->req.find(ticket);
  if (it == s->req.end()) {
    *done = 0;
    set_tl_error("hm_poll: unknown ticket");
    return HM_ENOTFOUND;
  }
  SrvReq& r = *it->second;
  if (!r.done) {
    *done = 0;
    return HM_EBUSY;
  }
  *done = 1;
  if (J_host && !r.J.empty()) std::copy(r.J.begin(), r.J.end(), J_host);
  if (q_host && !r.q.empty()) std::copy(r.q.begin(), r.q.end(), q_host);
  if (info) {
    info->iters = r.inner;
    info->outer_iters = r.rounds;
    info->matvecs = r.matvecs;
    info->rel_residual = r.rel_res;
    info->seconds = r.t_done - r.t_submit;
    info->bytes_moved = r.bytes;
  }
  if (latency) *latency = r.t_done - r.t_submit;
  const hm_status st = r.status;
  s->req.erase(it);
  return st;
}

hm_status hm_server_stats_get(hm_server* s, hm_server_stats* out) {
  if (!s || !out) return HM_EINVAL;
  std::lock_guard<std::mutex> lk(s->mu);
  *out = s->st;
  return HM_OK;
}

void hm_server_destroy(hm_server* s) {
  if (!s) return;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
    s->queue.clear();
  }
  s->cv.notify_all();
  s->acv.notify_all();
  if (s->worker.joinable()) s->worker.join();
  if (s->assembler.joinable()) s->assembler.join();
  (void)hipSetDevice(s->device);
  (void)hipStreamSynchronize(s->stream);
  if (s->actx.stream) (void)hipStreamSynchronize(s->actx.stream);
  s->cav.clear();
  s->req.clear();
  (void)hipStreamDestroy(s->stream);
  if (s->actx.stream) (void)hipStreamDestroy(s->actx.stream);
  delete s;
}

}  // extern "C"
