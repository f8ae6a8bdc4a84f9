// C ABI of the solver (declared in include/mx.h): context, state machine,
// operator assembly, ORAS set-up, and the pseudo-block flexible GMRES driver.
#include <algorithm>
#include <chrono>
#include <complex>
#include <functional>
#include <map>
#include <mutex>
#include <random>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "mx.h"
#include "block_lsq.h"
#include "host_mesh.h"
#include "mx_device.h"
#include "mx_kernels.h"
#include "tune_cache.h"

namespace mx {

thread_local std::string g_err;

// candidate panel groups of the factorisation autotuner (panels per
// trailing-update pass of the banded LU); the default without it
constexpr int kLuGroups[4] = {1, 2, 4, 8};
constexpr int kLuGroupDefault = 2;

int set_err(int code, const std::string& msg) {
  g_err = msg;
  return code;
}

int hip_fail(hipError_t e, const char* expr, const char* file, int line) {
  (void)hipGetLastError();
  g_err = std::string("HIP error ") + hipGetErrorString(e) + " in " + expr + " (" + file + ":" +
          std::to_string(line) + ")";
  return e == hipErrorOutOfMemory ? MX_ENOMEM : MX_EHIP;
}

template <typename T>
struct DBuf {
  T* p = nullptr;
  size_t n = 0;
  DBuf() = default;
  DBuf(const DBuf&) = delete;
  DBuf& operator=(const DBuf&) = delete;
  ~DBuf() { release(); }
  void release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    n = 0;
  }
  int alloc(size_t count) {
    if (p && count <= n) return MX_OK;
    release();
    if (count == 0) return MX_OK;
    hipError_t e = hipMalloc((void**)&p, count * sizeof(T));
    if (e != hipSuccess) {
      p = nullptr;
      (void)hipGetLastError();
      return set_err(MX_ENOMEM, "device allocation of " + std::to_string(count * sizeof(T)) + " bytes failed");
    }
    n = count;
    return MX_OK;
  }
  int upload(const std::vector<T>& v, hipStream_t s) {
    int rc = alloc(v.size());
    if (rc) return rc;
    if (!v.empty()) MX_HIP_CHECK(hipMemcpyAsync(p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, s));
    return MX_OK;
  }
};

bool is_device_ptr(const void* ptr) {
  if (!ptr) return false;
  hipPointerAttribute_t a;
  hipError_t e = hipPointerGetAttributes(&a, ptr);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  return a.type == hipMemoryTypeDevice;
}

// Fixed device buffer of mx_apply_preconditioner_noalloc: the restricted
// vectors of one preconditioner application live here instead of in memory
// the context allocates. Each GPU the library runs on holds its own copy.
// In host code `scratch` is only a handle for hipGetSymbolAddress; the
// device address is looked up once per device (scratch_address) and only
// that address is ever passed to kernels.
constexpr size_t kScratchBytes = size_t(64) << 20;
static __device__ __align__(256) char scratch[kScratchBytes];

std::mutex g_scratch_mu;
std::vector<void*> g_scratch_ptr;  // per device; nullptr until looked up

// device address of `scratch` on the current device `dev`
int scratch_address(int dev, void** out) {
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if ((int)g_scratch_ptr.size() <= dev) g_scratch_ptr.resize(dev + 1, nullptr);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)", __FILE__, __LINE__);
    if (!p) return set_err(MX_EHIP, "hipGetSymbolAddress(scratch) returned NULL");
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return MX_OK;
}

const double C0 = 299792458.0;
const double MU0 = 4.0e-7 * M_PI;

double2 csqrt_host(double2 z) {
  double r = std::hypot(z.x, z.y);
  double re = std::sqrt(0.5 * (r + z.x));
  double im = std::sqrt(std::max(0.5 * (r - z.x), 0.0));
  if (z.y < 0) im = -im;
  return make_double2(re, im);
}

__global__ void k_check_finite(int64_t n, const double2* v, int32_t* flag) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n && !(isfinite(v[i].x) && isfinite(v[i].y))) *flag = 1;
}
__global__ void k_set_g0(int m, int nrhs, const double* beta, double2* g) {
  int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (m + 1) * nrhs) return;
  g[idx] = idx < nrhs ? make_double2(beta[idx], 0.0) : make_double2(0.0, 0.0);
}
__global__ void k_zero_i32(int n, int32_t* a) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) a[i] = 0;
}
template <typename C>
__global__ void k_extract_local(int n, int N, const C* A, double2* out) {
  int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (idx >= (int64_t)n * n) return;
  int64_t i = idx / n, j = idx % n;
  out[idx] = to_c128(A[i * N + j]);
}

__global__ void k_scale_d(int n, double* x, double f) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) x[i] *= f;
}
__global__ void k_axpy_err(int64_t n, const double2* xs, const double2* x, const double2* mr, double2* t) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) t[i] = make_double2(xs[i].x - x[i].x - mr[i].x, xs[i].y - x[i].y - mr[i].y);
}

__global__ void k_sub(int64_t n, const double2* a, const double2* b, double2* o) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) o[i] = make_double2(a[i].x - b[i].x, a[i].y - b[i].y);
}
// theta_j = (Aq_j^H t_j) / ||Aq_j||^2; z += theta q, w += theta Aq
__global__ void k_theta_axpy(int64_t n, int nrhs, const double2* dot, const double* nrm, const double2* q,
                             const double2* aq, double2* z, double2* w) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  int j = (int)(i % nrhs);
  double d = nrm[j] * nrm[j];
  double2 th = d > 0 ? make_double2(dot[j].x / d, dot[j].y / d) : make_double2(0, 0);
  if (!(isfinite(th.x) && isfinite(th.y))) th = make_double2(0, 0);
  double2 a = q[i], b = aq[i];
  z[i] = make_double2(z[i].x + th.x * a.x - th.y * a.y, z[i].y + th.x * a.y + th.y * a.x);
  w[i] = make_double2(w[i].x + th.x * b.x - th.y * b.y, w[i].y + th.x * b.y + th.y * b.x);
}

struct SourceSet {
  std::vector<double> pos;   // cached copy to detect changes
  std::vector<double> mom;
  std::vector<int64_t> ptr;  // per point
  std::vector<int32_t> edge;
  std::vector<double2> val;
  bool same(const mx_sources* s) const {
    if (!s || (size_t)s->n * 3 != pos.size()) return false;
    return std::memcmp(pos.data(), s->pos, pos.size() * sizeof(double)) == 0 &&
           std::memcmp(mom.data(), s->moment, mom.size() * sizeof(double)) == 0;
  }
};

// HIP-event bracketing of kernel launches, per kernel class.
struct Profiler : KTimer {
  hipStream_t* stream = nullptr;
  bool on = false;
  std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> open, done;
  std::vector<hipEvent_t> pool;
  double ms[K_NCLASS] = {0};
  int64_t n[K_NCLASS] = {0};
  hipEvent_t get() {
    if (!pool.empty()) {
      hipEvent_t e = pool.back();
      pool.pop_back();
      return e;
    }
    hipEvent_t e = nullptr;
    (void)hipEventCreate(&e);
    return e;
  }
  void begin(int cls) override {
    if (!on) return;
    hipEvent_t a = get();
    (void)hipEventRecord(a, *stream);
    open.push_back({cls, {a, nullptr}});
  }
  void end(int cls) override {
    if (!on) return;
    for (size_t i = open.size(); i-- > 0;)
      if (open[i].first == cls) {
        hipEvent_t b = get();
        (void)hipEventRecord(b, *stream);
        open[i].second.second = b;
        done.push_back(open[i]);
        open.erase(open.begin() + i);
        break;
      }
    if (done.size() > 4096) resolve();
  }
  void resolve() {
    for (auto& d : done) {
      float t = 0;
      (void)hipEventSynchronize(d.second.second);
      (void)hipEventElapsedTime(&t, d.second.first, d.second.second);
      ms[d.first] += t;
      n[d.first] += 1;
      pool.push_back(d.second.first);
      pool.push_back(d.second.second);
    }
    done.clear();
  }
  void reset() {
    resolve();
    for (int i = 0; i < K_NCLASS; ++i) { ms[i] = 0; n[i] = 0; }
  }
  ~Profiler() {
    for (auto& d : done) { pool.push_back(d.second.first); pool.push_back(d.second.second); }
    for (auto e : pool) (void)hipEventDestroy(e);
  }
};

}  // namespace mx

using namespace mx;

struct mx_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  hipStream_t own_stream = nullptr;
  Profiler prof;
  // mesh
  Topology topo;
  bool have_mesh = false;
  DBuf<double> xyz;
  DBuf<int32_t> ts, col, csrc, bf_tet, bf_lf;
  DBuf<int64_t> row_ptr, cptr;
  // column windows of the operator's rows (SpMM variant 2; win_ok false when
  // some row has more columns than a window holds)
  ColWindows win;
  bool win_ok = false;
  DBuf<int32_t> win_row, win_cp, win_ucol;
  DBuf<uint8_t> win_lcol;
  // operator
  bool assembled = false;
  int eps_kind = 0;
  double freq = 0, k0 = 0, omega_mu0 = 0;
  double2 kb = {0, 0};
  DBuf<double2> eps, pool, val;
  size_t pool_filled = 0;
  // decomposition
  Decomposition dec;
  bool have_dec = false;
  DBuf<int32_t> dofs, Npad, order, trsm_order, if_tet, if_lf, lsrc, piv, status, pswap, perm, rowsrc, lpos,
      dense_edge;
  DBuf<int64_t> dof_ptr, mat_off, vec_off, ldest, lptr, pg_ptr, pg_row;
  // band bookkeeping of the factorisation (LuBand) and the triangular-solve
  // ranges derived from it; lu_tiles / trsm_tiles: 64x64 tile products of the
  // last factorisation and of one lower + upper solve per right-hand side
  DBuf<int32_t> ext_l, ext_u, tbox, trs_lo, trs_hi, band0, band_lim;
  DBuf<int64_t> tptr, band_work;
  int band_np = 0;
  int64_t lu_tiles = 0, trsm_tiles_l = 0, trsm_tiles_u = 0;
  DBuf<double> pg_w;
  std::vector<int32_t> Nsorted;
  DBuf<char> factors;
  int precision = MX_PREC_C128;
  bool local_ready = false, factored = false;
  int restart = 15, maxit = 2000;
  // wall time of the last mx_assemble / mx_setup_schwarz, device time of its LU
  double t_assemble = 0, t_setup = 0, t_lu = 0;
  hipEvent_t ev_lu[2] = {nullptr, nullptr};
  void* scratch_dev = nullptr;   // this device's address of the fixed scratch array
  // sources
  SourceSet tx, rx;
  DBuf<int32_t> s_edge, s_col, r_edge;
  DBuf<double2> s_val, r_val;
  DBuf<int64_t> r_ptr;
  // adjoint gradient
  bool have_forward = false;
  int last_ntx = 0, last_nrx = 0;
  double last_rtol = 1e-8;
  DBuf<int32_t> a_edge, a_col, t2e, v2t;
  DBuf<int64_t> v2t_ptr;
  DBuf<double2> a_val, U_fwd, gt, rt, gradv, keps;
  // learned coarse correction
  bool coarse_geom = false;      // lattices, P and G built for the current decomposition
  bool coarse_weights = false;   // network weights present
  bool coarse_use = false;       // opts.coarse of the last set-up
  bool coarse_off_now = false;   // disabled for the rest of the current solve (fallback)
  int coarse_fallbacks = 0;
  double sx = 1.0, sy = 1.0;     // input / output scales of the network
  DBuf<double2> qv, aq, tv, thdot;
  DBuf<double> thnrm, thtn;
  DBuf<char> xloc2;
  DBuf<float> cP, theta, gtheta, adam_m, adam_v, nbuf, gwork, dsX, dsY, cpart;
  DBuf<double> cbox, cG, cscale, cpdp, msepart;
  DBuf<int32_t> row_sub, edges_dev, cnbrs, bgraph, cflag;
  DBuf<int64_t> cnbr_ptr;
  int64_t nbuf_rows = 0;
  int64_t ds_graphs = 0, ds_cap = 0;
  int adam_t = 0;
  // workspace
  int ws_nrhs = 0, ws_m = 0;
  DBuf<double2> V, Z, x, b, r, H, sn, g, y, h1, h2, dotpart, S;
  DBuf<double> cs, bnorm, hn, beta, normpart, res;
  DBuf<int32_t> conv, kdone, flag;
  DBuf<char> xloc;
  int32_t* h_conv = nullptr;
  double* h_vec = nullptr;
  int32_t* h_kd = nullptr;
  int h_cap = 0;
  // waveguide ports and metallic walls
  std::vector<mx_port> ports;
  bool pec_walls = false;
  std::vector<int32_t> face_port;          // [nbf] port of each boundary face, -1: none
  std::vector<int32_t> pec_list;           // metallic edges
  std::vector<int64_t> pm_ptr;             // per port: moments int e_p.N_e over the port
  std::vector<int32_t> pm_edge;
  std::vector<double> pm_val, pm_norm;     // and int e_p.e_p
  DBuf<int32_t> pec_flag, pec_rows, pl_idx, pt_edge, pt_col;
  DBuf<int64_t> pl_ptr, pr_ptr;
  DBuf<double2> face_k, pt_val, pr_val;
  DBuf<int32_t> pr_edge;
  bool pec_local_ready = false;            // pl_ptr / pl_idx match the decomposition
  bool pool_envelope = false;  // factor pool zero outside the tiles ext_l / ext_u of its last factorisation
  // block FGMRES (mx_set_krylov): device blocks and pinned host staging
  int krylov_mode = MX_KRYLOV_PSEUDO_BLOCK;
  int64_t block_reorth = 0;                // one-pass block steps that took a second pass
  DBuf<double2> bw1, bw2, bpart, bH, bG, bT;
  double2* hb = nullptr;
  size_t hb_cap = 0;
  // Arnoldi steps captured as HIP graphs, one per step index k; valid while
  // the buffers, sizes and tolerance they were captured with are unchanged
  // autotuner: kernel variants picked by timing them on this problem
  bool autotune_on = true;
  uint64_t tune_key = 0;
  int tune_spmm = 0;           // 0: lanes per right-hand side, 1: broadcast entries, 2: LDS windows
  int tune_trsm_paired = 1;    // 1: size-paired workgroup order, 0: largest first
  int tune_trsm_cols = 32;     // right-hand-side columns per triangular-solve workgroup
  double tune_spmm_ms[3] = {0, 0, 0}, tune_trsm_ms[4] = {0, 0, 0, 0};
  // panels per trailing-update pass of the banded factorisation, picked by
  // timing whole factorisations at the first set-up of a shape bucket
  bool lu_autotune = true;
  uint64_t tune_lu_key = 0;
  int tune_lu_group = kLuGroupDefault;
  double tune_lu_ms[4] = {0, 0, 0, 0};
  bool tune_from_cache = false, tune_lu_from_cache = false;
  // every key this context has tuned, so that alternating shapes (phantoms
  // of a batch) are not timed again
  std::map<uint64_t, int> lu_tuned;
  std::map<uint64_t, std::vector<int>> solve_tuned;
  bool graphs_on = true;
  uint64_t g_sig = 0;         // signature of the buffers, sizes and tolerance captured
  std::vector<hipGraphExec_t> gexec;
  std::vector<char> gseen;
  void drop_graphs() {
    for (auto& e : gexec)
      if (e) (void)hipGraphExecDestroy(e);
    gexec.clear();
    gseen.clear();
    g_sig = 0;
  }
};

namespace {

#define CK(expr)                 \
  do {                           \
    int _rc = (expr);            \
    if (_rc != MX_OK) return _rc; \
  } while (0)

int use_device(mx_ctx* c) {
  MX_HIP_CHECK(hipSetDevice(c->device));
  return MX_OK;
}

// copies n elements between caller memory (host or device) and device memory
int copy_in(mx_ctx* c, void* dst_dev, const void* src, size_t bytes) {
  if (bytes == 0) return MX_OK;
  hipMemcpyKind k = is_device_ptr(src) ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
  MX_HIP_CHECK(hipMemcpyAsync(dst_dev, src, bytes, k, c->stream));
  return MX_OK;
}
int copy_out(mx_ctx* c, void* dst, const void* src_dev, size_t bytes) {
  if (bytes == 0 || !dst) return MX_OK;
  hipMemcpyKind k = is_device_ptr(dst) ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
  MX_HIP_CHECK(hipMemcpyAsync(dst, src_dev, bytes, k, c->stream));
  return MX_OK;
}
int sync(mx_ctx* c) {
  MX_HIP_CHECK(hipStreamSynchronize(c->stream));
  MX_HIP_CHECK(hipGetLastError());
  return MX_OK;
}

size_t elem_bytes(int prec) { return prec == MX_PREC_C64 ? sizeof(float2) : sizeof(double2); }

int ensure_host_pinned(mx_ctx* c, int n) {
  if (n <= c->h_cap) return MX_OK;
  if (c->h_conv) (void)hipHostFree(c->h_conv);
  if (c->h_vec) (void)hipHostFree(c->h_vec);
  if (c->h_kd) (void)hipHostFree(c->h_kd);
  c->h_conv = nullptr; c->h_vec = nullptr; c->h_kd = nullptr; c->h_cap = 0;
  MX_HIP_CHECK(hipHostMalloc((void**)&c->h_conv, n * sizeof(int32_t), hipHostMallocDefault));
  MX_HIP_CHECK(hipHostMalloc((void**)&c->h_vec, n * sizeof(double), hipHostMallocDefault));
  MX_HIP_CHECK(hipHostMalloc((void**)&c->h_kd, n * sizeof(int32_t), hipHostMallocDefault));
  c->h_cap = n;
  return MX_OK;
}

int ensure_workspace(mx_ctx* c, int nrhs, int m) {
  const int64_t ne = c->topo.ne;
  const size_t blk = (size_t)ne * nrhs;
  if (nrhs > 256) return set_err(MX_EINVAL, "at most 256 right-hand sides per solve");
  if (c->ws_nrhs != nrhs || c->ws_m != m) {
    CK(c->V.alloc(blk * (m + 1)));
    CK(c->Z.alloc(blk * m));
    CK(c->x.alloc(blk));
    CK(c->b.alloc(blk));
    CK(c->r.alloc(blk));
    CK(c->H.alloc((size_t)(m + 1) * m * nrhs));
    CK(c->sn.alloc((size_t)m * nrhs));
    CK(c->cs.alloc((size_t)m * nrhs));
    CK(c->g.alloc((size_t)(m + 1) * nrhs));
    CK(c->y.alloc((size_t)m * nrhs));
    CK(c->h1.alloc((size_t)(m + 1) * nrhs));
    CK(c->h2.alloc((size_t)(m + 1) * nrhs));
    CK(c->dotpart.alloc((size_t)dot_blocks(ne) * std::max(8, std::min(m + 1, cgs_fused_max())) * nrhs));
    CK(c->normpart.alloc((size_t)dot_blocks(ne) * nrhs));
    CK(c->bnorm.alloc(nrhs));
    CK(c->hn.alloc(nrhs));
    CK(c->beta.alloc(nrhs));
    CK(c->res.alloc(nrhs));
    CK(c->conv.alloc(nrhs));
    CK(c->kdone.alloc(nrhs));
    c->ws_nrhs = nrhs;
    c->ws_m = m;
  }
  if (c->have_dec) CK(c->xloc.alloc((size_t)c->dec.vec_off[c->dec.nsub] * nrhs * elem_bytes(c->precision)));
  CK(c->flag.alloc(4));
  CK(ensure_host_pinned(c, std::max(nrhs, 4)));
  return MX_OK;
}

// z = M^{-1} v (one ORAS application), v and z device blocks [ne][nrhs]

// ---------------------------------------------------------------------------
// learned coarse correction
// ---------------------------------------------------------------------------
constexpr int NCO = 192, NIN = 384, NW = 256;
// parameter layout (floats): W1 b1 W2 b2 W3 b3 W4 b4 Ws1 Wn1 b5 Ws2 Wn2 b6
struct NetLayout {
  int64_t W[4], b[4], Ws1, Wn1, b5, Ws2, Wn2, b6, total;
  NetLayout() {
    int64_t o = 0;
    for (int l = 0; l < 4; ++l) {
      W[l] = o;
      o += (int64_t)NW * (l == 0 ? NIN : NW);
      b[l] = o;
      o += NW;
    }
    Ws1 = o; o += (int64_t)NW * NW;
    Wn1 = o; o += (int64_t)NW * NW;
    b5 = o; o += NW;
    Ws2 = o; o += (int64_t)NIN * NW;
    Wn2 = o; o += (int64_t)NIN * NW;
    b6 = o; o += NIN;
    total = o;
  }
};
const NetLayout NL;

// activation buffers inside c->nbuf for `rows` rows
struct NetBufs {
  float *X, *Z[4], *H[4], *M4, *Z5, *H5, *M5, *OUT, *dOUT, *dH, *dZ, *dM, *T;
};
int net_bufs(mx_ctx* c, int64_t rows, NetBufs& B) {
  const int64_t per = rows * NW, pin = rows * NIN;
  const int64_t need = 2 * pin + 8 * per + 3 * per + 2 * pin + 4 * per;
  if (c->nbuf_rows < rows) {
    CK(c->nbuf.alloc((size_t)need));
    c->nbuf_rows = rows;
  }
  float* p = c->nbuf.p;
  B.X = p; p += pin;
  for (int l = 0; l < 4; ++l) { B.Z[l] = p; p += per; B.H[l] = p; p += per; }
  B.M4 = p; p += per; B.Z5 = p; p += per; B.H5 = p; p += per;
  B.M5 = p; p += per;
  B.OUT = p; p += pin; B.dOUT = p; p += pin;
  B.dH = p; p += per; B.dZ = p; p += per; B.dM = p; p += per; B.T = p; p += per;
  CK(c->gwork.alloc((size_t)16 * NIN * NIN));
  return MX_OK;
}

// network outputs B.OUT for inputs B.X (rows = ngraph * nsub)
void net_forward(mx_ctx* c, int ngraph, NetBufs& B) {
  const int nsub = c->dec.nsub;
  const int rows = ngraph * nsub;
  const float* th = c->theta.p;
  hipStream_t s = c->stream;
  const float* in = B.X;
  int K = NIN;
  for (int l = 0; l < 4; ++l) {
    launch_gemm(s, false, true, rows, NW, K, in, K, th + NL.W[l], K, B.H[l], NW, 0, th + NL.b[l], 1, B.Z[l], 1, 1,
                nullptr);
    in = B.H[l];
    K = NW;
  }
  launch_nbr_mean(s, ngraph, nsub, NW, c->cnbr_ptr.p, c->cnbrs.p, B.H[3], B.M4);
  launch_gemm(s, false, true, rows, NW, NW, B.H[3], NW, th + NL.Ws1, NW, B.H5, NW, 0, nullptr, 0, nullptr, 1, 1,
              nullptr);
  launch_gemm(s, false, true, rows, NW, NW, B.M4, NW, th + NL.Wn1, NW, B.H5, NW, 1, th + NL.b5, 1, B.Z5, 1, 1,
              nullptr);
  launch_nbr_mean(s, ngraph, nsub, NW, c->cnbr_ptr.p, c->cnbrs.p, B.H5, B.M5);
  launch_gemm(s, false, true, rows, NIN, NW, B.H5, NW, th + NL.Ws2, NW, B.OUT, NIN, 0, nullptr, 0, nullptr, 1, 1,
              nullptr);
  launch_gemm(s, false, true, rows, NIN, NW, B.M5, NW, th + NL.Wn2, NW, B.OUT, NIN, 1, th + NL.b6, 0, nullptr, 1, 1,
              nullptr);
}

// parameter gradient into c->gtheta from dOUT (after net_forward on the same rows)
void net_backward(mx_ctx* c, int ngraph, NetBufs& B) {
  const int nsub = c->dec.nsub;
  const int rows = ngraph * nsub;
  const float* th = c->theta.p;
  float* g = c->gtheta.p;
  hipStream_t s = c->stream;
  const int ns = 16;
  float* wk = c->gwork.p;
  // output layer
  launch_colsum(s, rows, NIN, B.dOUT, g + NL.b6);
  launch_gemm(s, true, false, NIN, NW, rows, B.dOUT, NIN, B.H5, NW, g + NL.Ws2, NW, 0, nullptr, 0, nullptr, 1, ns, wk);
  launch_gemm(s, true, false, NIN, NW, rows, B.dOUT, NIN, B.M5, NW, g + NL.Wn2, NW, 0, nullptr, 0, nullptr, 1, ns, wk);
  launch_gemm(s, false, false, rows, NW, NIN, B.dOUT, NIN, th + NL.Ws2, NW, B.dH, NW, 0, nullptr, 0, nullptr, 1, 1,
              nullptr);
  launch_gemm(s, false, false, rows, NW, NIN, B.dOUT, NIN, th + NL.Wn2, NW, B.dM, NW, 0, nullptr, 0, nullptr, 1, 1,
              nullptr);
  launch_nbr_mean_T(s, ngraph, nsub, NW, c->cnbr_ptr.p, c->cnbrs.p, B.dM, B.dH, 1);
  // message pass 1
  launch_gelu_back(s, (int64_t)rows * NW, B.dH, B.Z5, B.dZ);
  launch_colsum(s, rows, NW, B.dZ, g + NL.b5);
  launch_gemm(s, true, false, NW, NW, rows, B.dZ, NW, B.H[3], NW, g + NL.Ws1, NW, 0, nullptr, 0, nullptr, 1, ns, wk);
  launch_gemm(s, true, false, NW, NW, rows, B.dZ, NW, B.M4, NW, g + NL.Wn1, NW, 0, nullptr, 0, nullptr, 1, ns, wk);
  launch_gemm(s, false, false, rows, NW, NW, B.dZ, NW, th + NL.Ws1, NW, B.dH, NW, 0, nullptr, 0, nullptr, 1, 1,
              nullptr);
  launch_gemm(s, false, false, rows, NW, NW, B.dZ, NW, th + NL.Wn1, NW, B.dM, NW, 0, nullptr, 0, nullptr, 1, 1,
              nullptr);
  launch_nbr_mean_T(s, ngraph, nsub, NW, c->cnbr_ptr.p, c->cnbrs.p, B.dM, B.dH, 1);
  // MLP layers
  for (int l = 3; l >= 0; --l) {
    const int K = l == 0 ? NIN : NW;
    const float* a = l == 0 ? B.X : B.H[l - 1];
    launch_gelu_back(s, (int64_t)rows * NW, B.dH, B.Z[l], B.dZ);
    launch_colsum(s, rows, NW, B.dZ, g + NL.b[l]);
    launch_gemm(s, true, false, NW, K, rows, B.dZ, NW, a, K, g + NL.W[l], K, 0, nullptr, 0, nullptr, 1, ns, wk);
    if (l > 0)
      launch_gemm(s, false, false, rows, NW, NW, B.dZ, NW, th + NL.W[l], NW, B.dH, NW, 0, nullptr, 0, nullptr, 1, 1,
                  nullptr);
  }
}

void launch_sub(hipStream_t s, int64_t n, const double2* a, const double2* b, double2* o) {
  hipLaunchKernelGGL(k_sub, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n, a, b, o);
}
void launch_theta_axpy(hipStream_t s, int64_t n, int nrhs, const double2* dot, const double* nrm, const double2* q,
                       const double2* aq, double2* z, double2* w) {
  hipLaunchKernelGGL(k_theta_axpy, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n, nrhs, dot, nrm, q, aq, z, w);
}

void launch_scale_rhs_norm(mx_ctx* c, int nrhs) {
  hipLaunchKernelGGL(k_scale_d, dim3((unsigned)((nrhs + 255) / 256)), dim3(256), 0, c->stream, nrhs, c->cscale.p,
                     1.0 / std::sqrt((double)c->topo.ne));
}

// network correction of one preconditioner application (after the local solves)
template <typename C>
void coarse_correct(mx_ctx* c, const double2* v, C* xl, int nrhs) {
  const Decomposition& D = c->dec;
  hipStream_t s = c->stream;
  NetBufs B;
  if (net_bufs(c, (int64_t)nrhs * D.nsub, B) != MX_OK) return;
  // s_j = ||v_j|| / sqrt(ne)
  launch_norm(s, c->topo.ne, nrhs, v, c->normpart.p, c->cscale.p);
  launch_scale_rhs_norm(c, nrhs);
  launch_pool(s, D.nsub, c->dof_ptr.p, c->dofs.p, c->cP.p, nullptr, v, nrhs, c->cscale.p, B.X, c->cpart.p);
  launch_scale_f(s, (int64_t)nrhs * D.nsub * NIN, B.X, (float)(1.0 / c->sx));
  net_forward(c, nrhs, B);
  launch_nonfinite(s, (int64_t)nrhs * D.nsub * NIN, B.OUT, c->cflag.p);
  launch_coarse_apply<C>(s, D.dof_ptr[D.nsub], c->lpos.p, c->dof_ptr.p, c->vec_off.p, c->cP.p, B.OUT, D.nsub,
                         nrhs, c->cscale.p, (float)c->sy, xl);
}

// z = M^{-1} v; with the learned term active it is added to z, or, when q is
// given, returned separately in q (z then holds plain ORAS)
// local: the restricted-vector buffer ([sum N_i][nrhs] in the factor
// precision); NULL uses the context's own, any other buffer runs the same
// kernels without the profiler (no event is created or recorded); z2, ld2:
// an optional second destination of z (row stride ld2)
template <typename R>
void apply_precond_t(mx_ctx* c, const double2* v, double2* z, int nrhs, double2* q = nullptr, void* local = nullptr,
                     double2* z2 = nullptr, int64_t ld2 = 0) {
  typedef C_t<R> C;
  const Decomposition& D = c->dec;
  const int64_t nrows = D.vec_off[D.nsub];
  C* xl = local ? (C*)local : (C*)c->xloc.p;
  KTimer* tm = local ? nullptr : &c->prof;
  if (tm) tm->begin(K_RESTRICT);
  launch_restrict<C>(c->stream, nrows, c->rowsrc.p, v, xl, nrhs);
  if (tm) tm->end(K_RESTRICT);
  launch_trsm<R>(c->stream, (const C*)c->factors.p, c->mat_off.p, c->Npad.p, c->vec_off.p,
                 c->tune_trsm_paired ? c->trsm_order.p : c->order.p, xl, D.nsub, nrhs, c->trs_lo.p, c->trs_hi.p,
                 c->band_np, c->tune_trsm_cols, tm);
  const bool coarse = !local && c->coarse_use && !c->coarse_off_now && c->coarse_geom && c->coarse_weights;
  C* xq = nullptr;
  if (coarse) {
    c->prof.begin(K_COARSE);
    if (q) {
      // learned term in its own local buffer, prolonged separately into q
      xq = (C*)c->xloc2.p;
      launch_fill_zero<C>(c->stream, nrows * nrhs, xq);
      coarse_correct<C>(c, v, xq, nrhs);
    } else {
      coarse_correct<C>(c, v, xl, nrhs);
    }
    c->prof.end(K_COARSE);
  }
  if (tm) tm->begin(K_PROLONG);
  launch_prolong<C>(c->stream, c->topo.ne, c->pg_ptr.p, c->pg_row.p, c->pg_w.p, xl, z, nrhs, z2, ld2);
  if (xq) launch_prolong<C>(c->stream, c->topo.ne, c->pg_ptr.p, c->pg_row.p, c->pg_w.p, xq, q, nrhs);
  if (tm) tm->end(K_PROLONG);
}

int apply_precond(mx_ctx* c, const double2* v, double2* z, int nrhs, double2* q = nullptr, void* local = nullptr,
                  double2* z2 = nullptr, int64_t ld2 = 0) {
  if (c->precision == MX_PREC_C64)
    apply_precond_t<float>(c, v, z, nrhs, q, local, z2, ld2);
  else
    apply_precond_t<double>(c, v, z, nrhs, q, local, z2, ld2);
  MX_HIP_CHECK(hipGetLastError());
  return MX_OK;
}

SpmmWindows windows(const mx_ctx* c) {
  if (!c->win_ok) return SpmmWindows{0, nullptr, nullptr, nullptr, nullptr};
  return SpmmWindows{(int32_t)(c->win.row.size() - 1), c->win_row.p, c->win_cp.p, c->win_ucol.p, c->win_lcol.p};
}

int spmm(mx_ctx* c, const double2* X, double2* Y, int nrhs) {
  c->prof.begin(K_SPMM);
  const SpmmWindows w = windows(c);
  launch_spmm(c->stream, c->topo.ne, c->row_ptr.p, c->col.p, c->val.p, X, Y, nrhs, c->tune_spmm, &w);
  c->prof.end(K_SPMM);
  MX_HIP_CHECK(hipGetLastError());
  return MX_OK;
}

bool learned_ready(const mx_ctx* c) { return c->coarse_use && c->coarse_geom && c->coarse_weights; }

// buffers of precond_learned for nrhs columns
int ensure_learned_ws(mx_ctx* c, int nrhs) {
  const size_t blk = (size_t)c->topo.ne * nrhs;
  CK(c->qv.alloc(blk));
  CK(c->aq.alloc(blk));
  CK(c->tv.alloc(blk));
  CK(c->thdot.alloc(nrhs));
  CK(c->thnrm.alloc(nrhs));
  CK(c->thtn.alloc(nrhs));
  CK(c->xloc2.alloc((size_t)c->dec.vec_off[c->dec.nsub] * nrhs * elem_bytes(c->precision)));
  CK(c->xloc.alloc((size_t)c->dec.vec_off[c->dec.nsub] * nrhs * elem_bytes(c->precision)));
  CK(c->dotpart.alloc((size_t)dot_blocks(c->topo.ne) * 8 * nrhs));
  CK(c->normpart.alloc((size_t)dot_blocks(c->topo.ne) * nrhs));
  return MX_OK;
}

// The preconditioner with the learned term as FGMRES uses it:
// z = M^{-1} v + theta_j q_j, one weight per column minimising ||v_j - A z_j||
// (theta_j = (A q_j)^H t_j / ||A q_j||^2 with t = v - A M^{-1} v), and
// w = A z. Scratch: qv (q), aq (A q), tv (t); thdot / thnrm / thtn keep
// (A q)^H t, ||A q|| and ||t|| per column for the judge.
int precond_learned(mx_ctx* c, const double2* v, double2* z, double2* w, int nrhs) {
  hipStream_t s = c->stream;
  const int64_t ne = c->topo.ne;
  const int64_t blk = ne * (int64_t)nrhs;
  CK(apply_precond(c, v, z, nrhs, c->qv.p));
  CK(spmm(c, z, w, nrhs));
  CK(spmm(c, c->qv.p, c->aq.p, nrhs));
  launch_sub(s, blk, v, w, c->tv.p);
  launch_dot(s, ne, nrhs, c->aq.p, blk, 1, c->tv.p, c->dotpart.p, c->thdot.p);
  launch_norm(s, ne, nrhs, c->aq.p, c->normpart.p, c->thnrm.p);
  launch_norm(s, ne, nrhs, c->tv.p, c->normpart.p, c->thtn.p);
  launch_theta_axpy(s, blk, nrhs, c->thdot.p, c->thnrm.p, c->qv.p, c->aq.p, z, w);
  MX_HIP_CHECK(hipGetLastError());
  return MX_OK;
}

// Right-preconditioned pseudo-block FGMRES on b (device) -> x (device, ctx->x).
// on_cycle (optional) runs at the start of every restart cycle with the
// current iterate in c->x and its true residual in c->r.
// Autotuner: at the first solve of a problem shape (edges, non-zeros,
// subdomains, factor entries, precision, right-hand sides) every candidate
// variant of the SpMM and of the triangular-solve workgroup order is run on
// this problem's own data (X = b; the restricted b) and timed with HIP
// events; the fastest is kept for the following solves.
// triangular-solve shapes: workgroup order (largest first / size-paired) x
// right-hand-side columns per workgroup (32 / 16)
template <typename R>
int autotune_trsm(mx_ctx* c, int nrhs, hipEvent_t e0, hipEvent_t e1) {
  typedef C_t<R> C;
  const Decomposition& D = c->dec;
  C* xl = (C*)c->xloc.p;
  launch_restrict<C>(c->stream, D.vec_off[D.nsub], c->rowsrc.p, c->b.p, xl, nrhs);
  int best = 0;
  for (int v = 0; v < 4; ++v) {
    const int32_t* ord = (v & 1) ? c->trsm_order.p : c->order.p;
    const int cols = v < 2 ? 32 : 16;
    launch_trsm<R>(c->stream, (const C*)c->factors.p, c->mat_off.p, c->Npad.p, c->vec_off.p, ord, xl, D.nsub, nrhs,
                   c->trs_lo.p, c->trs_hi.p, c->band_np, cols, nullptr);
    MX_HIP_CHECK(hipEventRecord(e0, c->stream));
    launch_trsm<R>(c->stream, (const C*)c->factors.p, c->mat_off.p, c->Npad.p, c->vec_off.p, ord, xl, D.nsub, nrhs,
                   c->trs_lo.p, c->trs_hi.p, c->band_np, cols, nullptr);
    MX_HIP_CHECK(hipEventRecord(e1, c->stream));
    MX_HIP_CHECK(hipEventSynchronize(e1));
    float ms = 0;
    MX_HIP_CHECK(hipEventElapsedTime(&ms, e0, e1));
    c->tune_trsm_ms[v] = ms;
    if (ms < c->tune_trsm_ms[best]) best = v;
  }
  c->tune_trsm_paired = best & 1;
  c->tune_trsm_cols = best < 2 ? 32 : 16;
  return MX_OK;
}

int autotune(mx_ctx* c, int nrhs) {
  if (!c->autotune_on) return MX_OK;
  uint64_t key = 1469598103934665603ull;
  auto mixv = [&](int64_t v) { key = (key ^ (uint64_t)v) * 1099511628211ull; };
  mixv(c->topo.ne);
  mixv((int64_t)c->col.n);
  mixv(c->dec.nsub);
  mixv(c->dec.mat_off.empty() ? 0 : c->dec.mat_off.back());
  mixv(c->precision);
  mixv(nrhs);
  if (key == c->tune_key) return MX_OK;
  const auto seen = c->solve_tuned.find(key);
  if (c->factored && seen != c->solve_tuned.end() && !(seen->second[0] == 2 && !c->win_ok)) {
    c->tune_spmm = seen->second[0];
    c->tune_trsm_paired = seen->second[1];
    c->tune_trsm_cols = seen->second[2];
    c->tune_key = key;
    return MX_OK;
  }
  char hex[32];
  std::snprintf(hex, sizeof hex, "%016llx", (unsigned long long)key);
  const std::string ckey = std::string("solve:") + hex;
  TuneFields tf;
  if (c->factored && tune_cache_get(ckey, tf) && tf.count("spmm") && tf.count("trsm_paired") && tf.count("trsm_cols")) {
    const long long v = tf["spmm"], pr = tf["trsm_paired"], tc = tf["trsm_cols"];
    if (v >= 0 && v <= 2 && !(v == 1 && nrhs > 32) && !(v == 2 && !c->win_ok) && (pr == 0 || pr == 1) &&
        (tc == 16 || tc == 32)) {
      c->tune_spmm = (int)v;
      c->tune_trsm_paired = (int)pr;
      c->tune_trsm_cols = (int)tc;
      for (double& t : c->tune_spmm_ms) t = 0;
      for (double& t : c->tune_trsm_ms) t = 0;
      c->tune_from_cache = true;
      c->tune_key = key;
      c->solve_tuned[key] = {c->tune_spmm, c->tune_trsm_paired, c->tune_trsm_cols};
      return MX_OK;
    }
  }
  hipEvent_t e0 = nullptr, e1 = nullptr;
  MX_HIP_CHECK(hipEventCreate(&e0));
  MX_HIP_CHECK(hipEventCreate(&e1));
  const int64_t ne = c->topo.ne;
  int rc = MX_OK;
  const SpmmWindows w = windows(c);
  for (int v = 0; v < 3 && rc == MX_OK; ++v) {
    if ((v == 1 && nrhs > 32) || (v == 2 && !c->win_ok)) {
      c->tune_spmm_ms[v] = 1e30;
      continue;
    }
    launch_spmm(c->stream, ne, c->row_ptr.p, c->col.p, c->val.p, c->b.p, c->r.p, nrhs, v, &w);
    hipError_t e = hipEventRecord(e0, c->stream);
    for (int it = 0; it < 3; ++it)
      launch_spmm(c->stream, ne, c->row_ptr.p, c->col.p, c->val.p, c->b.p, c->r.p, nrhs, v, &w);
    if (e == hipSuccess) e = hipEventRecord(e1, c->stream);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float ms = 0;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    if (e != hipSuccess) rc = hip_fail(e, "autotune spmm", __FILE__, __LINE__);
    c->tune_spmm_ms[v] = ms / 3;
  }
  if (rc == MX_OK) {
    c->tune_spmm = 0;
    for (int v = 1; v < 3; ++v)
      if (c->tune_spmm_ms[v] < c->tune_spmm_ms[c->tune_spmm]) c->tune_spmm = v;
  }
  if (rc == MX_OK && c->factored)
    rc = c->precision == MX_PREC_C64 ? autotune_trsm<float>(c, nrhs, e0, e1) : autotune_trsm<double>(c, nrhs, e0, e1);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc == MX_OK) {
    c->tune_key = key;
    c->tune_from_cache = false;
    if (c->factored) c->solve_tuned[key] = {c->tune_spmm, c->tune_trsm_paired, c->tune_trsm_cols};
    if (c->factored)
      tune_cache_put(ckey, {{"spmm", c->tune_spmm}, {"trsm_paired", c->tune_trsm_paired},
                            {"trsm_cols", c->tune_trsm_cols}});
  }
  return rc;
}

// FNV-1a over every pointer, size and scalar a captured Arnoldi step bakes in
uint64_t step_signature(const mx_ctx* c, int nrhs, int m, double rtol) {
  uint64_t h = 1469598103934665603ull;
  auto mix = [&](const void* p, size_t n) {
    const unsigned char* b = (const unsigned char*)p;
    for (size_t i = 0; i < n; ++i) h = (h ^ b[i]) * 1099511628211ull;
  };
  auto val = [&](auto v) { mix(&v, sizeof(v)); };
  const void* ptrs[] = {c->V.p, c->Z.p, c->xloc.p, c->factors.p, c->val.p, c->row_ptr.p, c->col.p,
                        c->rowsrc.p, c->trsm_order.p, c->mat_off.p, c->Npad.p, c->vec_off.p, c->pg_ptr.p,
                        c->pg_row.p, c->pg_w.p, c->dotpart.p, c->normpart.p, c->h1.p, c->h2.p, c->hn.p, c->H.p,
                        c->cs.p, c->sn.p, c->g.p, c->bnorm.p, c->conv.p, c->kdone.p, c->res.p, c->trs_lo.p,
                        c->trs_hi.p, c->win_row.p, c->win_cp.p, c->win_ucol.p, c->win_lcol.p};
  mix(ptrs, sizeof(ptrs));
  val(c->topo.ne);
  val(c->win_ok);
  val(c->win.row.size());
  val(c->dec.nsub);
  val(c->dec.ncolour);
  val(c->precision);
  val(c->tune_spmm);
  val(c->tune_trsm_paired);
  val(c->tune_trsm_cols);
  val(nrhs);
  val(m);
  val(rtol);
  if (!c->dec.vec_off.empty()) val(c->dec.vec_off.back());
  mix(c->dec.pcol_ptr.data(), c->dec.pcol_ptr.size() * sizeof(int64_t));
  return h;
}

// ---------------------------------------------------------------------------
// Block FGMRES: one block Krylov space shared by all right-hand sides
// (block Arnoldi, Saad, Iterative Methods for Sparse Linear Systems, Sec. 6.12)
// ---------------------------------------------------------------------------
typedef std::complex<double> cd;
constexpr int kBlockFallback = 1000;  // internal: run the pseudo-block solver instead

// G = R^H R for the Hermitian Gram matrix G (s x s, row-major) of a block,
// through the Cholesky factor of D^-1 G D^-1 (D = diag(G)^(1/2)), so that the
// column scales of the block do not enter the rank test: false when a scaled
// pivot is not above tol (the block has numerical rank below s).
bool gram_cholesky(const double2* G, int s, std::vector<cd>& R, double tol, double* min_pivot = nullptr) {
  std::vector<double> d(s);
  for (int i = 0; i < s; ++i) {
    const double g = G[(size_t)i * s + i].x;
    if (!(g > 0) || !std::isfinite(g)) return false;
    d[i] = std::sqrt(g);
  }
  std::vector<cd> L((size_t)s * s, 0.0);
  double pmin = 1.0;
  for (int j = 0; j < s; ++j) {
    double piv = G[(size_t)j * s + j].x / (d[j] * d[j]);
    for (int k = 0; k < j; ++k) piv -= std::norm(L[(size_t)j * s + k]);
    if (!(piv > tol)) return false;
    pmin = std::min(pmin, piv);
    const double ljj = std::sqrt(piv);
    L[(size_t)j * s + j] = ljj;
    for (int i = j + 1; i < s; ++i) {
      const double2 g = G[(size_t)i * s + j];
      cd v = cd(g.x, g.y) / (d[i] * d[j]);
      for (int k = 0; k < j; ++k) v -= L[(size_t)i * s + k] * std::conj(L[(size_t)j * s + k]);
      L[(size_t)i * s + j] = v / ljj;
    }
  }
  R.assign((size_t)s * s, 0.0);
  for (int i = 0; i < s; ++i)
    for (int j = i; j < s; ++j) R[(size_t)i * s + j] = std::conj(L[(size_t)j * s + i]) * d[j];
  if (min_pivot) *min_pivot = pmin;
  return true;
}

// T = R^-1 for upper triangular R (row-major)
void upper_inverse(const std::vector<cd>& R, int s, double2* T) {
  std::vector<cd> X((size_t)s * s, 0.0);
  for (int j = 0; j < s; ++j) {
    X[(size_t)j * s + j] = 1.0 / R[(size_t)j * s + j];
    for (int i = j - 1; i >= 0; --i) {
      cd v = 0;
      for (int k = i + 1; k <= j; ++k) v += R[(size_t)i * s + k] * X[(size_t)k * s + j];
      X[(size_t)i * s + j] = -v / R[(size_t)i * s + i];
    }
  }
  for (size_t e = 0; e < X.size(); ++e) T[e] = make_double2(X[e].real(), X[e].imag());
}

int ensure_block_host(mx_ctx* c, size_t n) {
  if (n <= c->hb_cap) return MX_OK;
  if (c->hb) (void)hipHostFree(c->hb);
  c->hb = nullptr;
  c->hb_cap = 0;
  MX_HIP_CHECK(hipHostMalloc((void**)&c->hb, n * sizeof(double2), hipHostMallocDefault));
  c->hb_cap = n;
  return MX_OK;
}

// W = Q R by Cholesky QR (W, tmp, out: s columns, row stride ld), applied a
// second time unless the scaled block is well conditioned: Q written to out,
// tmp scratch, R (upper, row-major) on the host. ok = false when the block
// has numerical rank below s (out is then not written).
// G1 (host, optional): W^H W when the caller already has it. out2, ld2
// (optional): a second destination of Q (the block's place in the basis).
int cholqr2(mx_ctx* c, int s, const double2* W, double2* tmp, double2* out, int64_t ld, std::vector<cd>& R,
            bool& ok, const double2* G1 = nullptr, double2* out2 = nullptr, int64_t ld2 = 0) {
  const int64_t ne = c->topo.ne;
  hipStream_t st = c->stream;
  const size_t ss = (size_t)s * s;
  double2* hG = c->hb;
  double2* hT = c->hb + ss;
  std::vector<cd> R1, R2;
  // pass 1 (rank test on the scaled Gram matrix; 1e-14 keeps cond(W D^-1) below ~1e7)
  if (G1) {
    if (G1 != hG) std::memcpy(hG, G1, ss * sizeof(double2));
  } else {
    launch_bdot(st, ne, s, s, W, ld, W, ld, c->bpart.p, c->bG.p);
    MX_HIP_CHECK(hipMemcpyAsync(hG, c->bG.p, ss * sizeof(double2), hipMemcpyDeviceToHost, st));
    CK(sync(c));
  }
  double pmin = 0;
  ok = gram_cholesky(hG, s, R1, 1e-14, &pmin);
  if (!ok) return MX_OK;
  upper_inverse(R1, s, hT);
  MX_HIP_CHECK(hipMemcpyAsync(c->bT.p, hT, ss * sizeof(double2), hipMemcpyHostToDevice, st));
  if (pmin >= 1e-4) {
    // the scaled block has condition number below ~100: one pass leaves Q
    // orthonormal to ~1e-12, the second is skipped
    launch_bupd(st, ne, s, s, W, ld, c->bT.p, nullptr, 0, out, ld, 1.0, 0.0, out2, ld2);
    MX_HIP_CHECK(hipGetLastError());
    R = R1;
    return MX_OK;
  }
  launch_bupd(st, ne, s, s, W, ld, c->bT.p, nullptr, 0, tmp, ld, 1.0, 0.0);
  // pass 2 on the (nearly orthonormal) first factor
  launch_bdot(st, ne, s, s, tmp, ld, tmp, ld, c->bpart.p, c->bG.p);
  MX_HIP_CHECK(hipMemcpyAsync(hG, c->bG.p, ss * sizeof(double2), hipMemcpyDeviceToHost, st));
  CK(sync(c));
  ok = gram_cholesky(hG, s, R2, 1e-10);
  if (!ok) return MX_OK;
  upper_inverse(R2, s, hT);
  MX_HIP_CHECK(hipMemcpyAsync(c->bT.p, hT, ss * sizeof(double2), hipMemcpyHostToDevice, st));
  launch_bupd(st, ne, s, s, tmp, ld, c->bT.p, nullptr, 0, out, ld, 1.0, 0.0, out2, ld2);
  MX_HIP_CHECK(hipGetLastError());
  R.assign(ss, 0.0);  // R = R2 R1
  for (int i = 0; i < s; ++i)
    for (int j = i; j < s; ++j) {
      cd v = 0;
      for (int k = i; k <= j; ++k) v += R2[(size_t)i * s + k] * R1[(size_t)k * s + j];
      R[(size_t)i * s + j] = v;
    }
  return MX_OK;
}

// Block right-preconditioned FGMRES on b (device) -> x (device, ctx->x) with
// the one-level preconditioner. The right-hand sides are split into groups of
// at most 32 columns; every group has its own block Krylov space, and the
// groups advance in lockstep so that the preconditioner and the operator are
// applied to the whole width at once. Layout: a group's basis blocks
// V_0..V_m sit side by side, row r of the basis holding (m+1)s values
// (ld (m+1)s), its preconditioned blocks Z_0..Z_{m-1} likewise (ld ms), so
// that V^H W, W - V H and X + Z Y are single tall-skinny products. Each step
// of a group: Z_k = M^-1 V_k, W = A Z_k, one pass of block classical
// Gram-Schmidt (a second one when W lay almost entirely in the basis),
// W = V_{k+1} R_{k+1} by Cholesky QR (twice unless well conditioned).
// from_x: start from the iterate in ctx->x instead of 0. Returns
// kBlockFallback (x unchanged) when a right-hand side is zero or a residual
// block has numerical rank below its width at the first cycle.
int block_fgmres(mx_ctx* c, int S, double rtol, mx_solve_info* info, bool from_x = false) {
  const bool two_pass = c->krylov_mode == MX_KRYLOV_BLOCK_CGS2;
  const int m = c->ws_m;
  const int64_t ne = c->topo.ne;
  const int64_t blk = ne * (int64_t)S;
  const int G = (S + 31) / 32;
  std::vector<int> g0(G + 1), gs(G);
  for (int g = 0; g <= G; ++g) g0[g] = (int)((int64_t)g * S / G);
  for (int g = 0; g < G; ++g) gs[g] = g0[g + 1] - g0[g];
  hipStream_t st = c->stream;
  auto t0 = std::chrono::steady_clock::now();
  CK(autotune(c, S));
  const int64_t LVmax = (int64_t)(m + 1) * 32;
  CK(c->bw1.alloc(blk));
  CK(c->bw2.alloc(blk));
  CK(c->bpart.alloc(block_partial_max((int)LVmax, 32)));
  CK(c->bH.alloc(LVmax * 32));
  CK(c->bG.alloc(32 * 32));
  CK(c->bT.alloc(32 * 32));
  CK(ensure_block_host(c, 2 * 32 * 32 + 2 * (size_t)LVmax * 32));
  double2* hh1 = c->hb + 2 * 32 * 32;
  double2* hh2 = hh1 + (size_t)LVmax * 32;
  launch_norm(st, ne, S, c->b.p, c->normpart.p, c->bnorm.p);
  MX_HIP_CHECK(hipMemcpyAsync(c->h_vec, c->bnorm.p, S * sizeof(double), hipMemcpyDeviceToHost, st));
  CK(sync(c));
  std::vector<double> bn(S), rr(S);
  for (int j = 0; j < S; ++j) {
    bn[j] = c->h_vec[j];
    if (!(bn[j] > 0)) return kBlockFallback;
  }
  c->coarse_off_now = true;  // the learned term is not used with the block solver
  if (from_x) {  // continue from the current iterate
    CK(spmm(c, c->x.p, c->r.p, S));
    launch_bminus(st, blk, c->b.p, c->r.p);
  } else {
    launch_fill_zero<double2>(st, blk, c->x.p);
    MX_HIP_CHECK(hipMemcpyAsync(c->r.p, c->b.p, blk * sizeof(double2), hipMemcpyDeviceToDevice, st));
  }
  auto true_residual = [&]() -> int {
    launch_norm(st, ne, S, c->r.p, c->normpart.p, c->beta.p);
    MX_HIP_CHECK(hipMemcpyAsync(c->h_vec, c->beta.p, S * sizeof(double), hipMemcpyDeviceToHost, st));
    CK(sync(c));
    for (int j = 0; j < S; ++j) rr[j] = c->h_vec[j] / bn[j];
    return MX_OK;
  };
  CK(true_residual());
  std::vector<BlockLsq> ls(G);
  std::vector<char> active(G, 1), running(G, 0);
  std::vector<int> kk(G, 0), steps(G, 0);
  auto Vg = [&](int g) { return c->V.p + (int64_t)(m + 1) * ne * g0[g]; };
  auto Zg = [&](int g) { return c->Z.p + (int64_t)m * ne * g0[g]; };
  int total = 0, cycles = 0, rc = MX_OK;
  std::vector<cd> Rk, P;
  for (;;) {
    int nact = 0;
    for (int g = 0; g < G; ++g) {
      double worst = 0;
      for (int j = g0[g]; j < g0[g + 1]; ++j) worst = std::max(worst, rr[j]);
      active[g] = active[g] && worst > rtol;
      nact += active[g];
    }
    if (nact == 0) break;
    if (total >= c->maxit) {
      rc = set_err(MX_ENOTCONV, "block FGMRES reached maxit=" + std::to_string(c->maxit));
      break;
    }
    // R_g = V_0 S0 for every unfinished group
    c->prof.begin(K_CGS);
    for (int g = 0; g < G; ++g) {
      running[g] = 0;
      kk[g] = 0;
      if (!active[g]) continue;
      bool ok = false;
      CK(cholqr2(c, gs[g], c->r.p + g0[g], c->bw1.p + g0[g], c->bw2.p + g0[g], S, Rk, ok, nullptr, Vg(g),
                 (int64_t)(m + 1) * gs[g]));
      if (!ok) {
        c->prof.end(K_CGS);
        if (total > 0) return set_err(MX_ENOTCONV, "block FGMRES: a residual block lost rank");
        return kBlockFallback;
      }
      ls[g].reset(gs[g], m, Rk);
      running[g] = 1;
    }
    c->prof.end(K_CGS);
    for (int k = 0; k < m && total < c->maxit; ++k) {
      bool any = false;
      for (int g = 0; g < G; ++g) any = any || running[g];
      if (!any) break;
      // bw2: V_k of every group; bw1: Z_k; r: W (whole width)
      if (G == 1) {  // one group: the preconditioner writes Z_k into the basis as well
        CK(apply_precond(c, c->bw2.p, c->bw1.p, S, nullptr, nullptr, Zg(0) + (int64_t)k * gs[0], (int64_t)m * gs[0]));
      } else {
        CK(apply_precond(c, c->bw2.p, c->bw1.p, S));
        for (int g = 0; g < G; ++g)
          if (running[g])
            launch_bcopy(st, ne, gs[g], c->bw1.p + g0[g], S, Zg(g) + (int64_t)k * gs[g], (int64_t)m * gs[g]);
      }
      CK(spmm(c, c->bw1.p, c->r.p, S));
      c->prof.begin(K_CGS);
      for (int g = 0; g < G; ++g) {
        if (!running[g]) continue;
        const int s = gs[g];
        const int64_t LV = (int64_t)(m + 1) * s;
        double2* W = c->r.p + g0[g];
        const int ka = (k + 1) * s;
        const size_t ss = (size_t)s * s;
        bool reorth = false, ok = false;
        launch_bdot(st, ne, ka, s, Vg(g), LV, W, S, c->bpart.p, c->bH.p);
        MX_HIP_CHECK(hipMemcpyAsync(hh1, c->bH.p, (size_t)ka * s * sizeof(double2), hipMemcpyDeviceToHost, st));
        if (two_pass) {
          launch_bupd(st, ne, ka, s, Vg(g), LV, c->bH.p, W, S, W, S, -1.0, 1.0);
          launch_bdot(st, ne, ka, s, Vg(g), LV, W, S, c->bpart.p, c->bH.p);
          MX_HIP_CHECK(hipMemcpyAsync(hh2, c->bH.p, (size_t)ka * s * sizeof(double2), hipMemcpyDeviceToHost, st));
          launch_bupd(st, ne, ka, s, Vg(g), LV, c->bH.p, W, S, W, S, -1.0, 1.0);
          CK(cholqr2(c, s, W, c->bw1.p + g0[g], c->bw2.p + g0[g], S, Rk, ok, nullptr, Vg(g) + (int64_t)(k + 1) * s,
                     LV));
        } else {
          // one projection pass, repeated only when W lay almost entirely in
          // the basis (its column norms fell by more than 1e4 in the pass, so
          // that one pass leaves a loss of orthogonality above ~1e-12); then
          // Cholesky QR (twice unless well conditioned)
          // (||W_j||^2 = ||W'_j||^2 + ||H1_j||^2 for the orthonormal basis)
          double2* hG1 = c->hb;
          launch_bupd(st, ne, ka, s, Vg(g), LV, c->bH.p, W, S, W, S, -1.0, 1.0);
          launch_bdot(st, ne, s, s, W, S, W, S, c->bpart.p, c->bG.p);
          MX_HIP_CHECK(hipMemcpyAsync(hG1, c->bG.p, ss * sizeof(double2), hipMemcpyDeviceToHost, st));
          CK(sync(c));
          double rho = 1.0;
          for (int j = 0; j < s; ++j) {
            double h2 = 0;
            for (int a = 0; a < ka; ++a) {
              const double2 h = hh1[(size_t)a * s + j];
              h2 += h.x * h.x + h.y * h.y;
            }
            const double w2 = hG1[(size_t)j * s + j].x;
            rho = std::min(rho, w2 / (w2 + h2));
          }
          reorth = !(rho >= 1e-8);
          if (reorth) {
            ++c->block_reorth;
            launch_bdot(st, ne, ka, s, Vg(g), LV, W, S, c->bpart.p, c->bH.p);
            MX_HIP_CHECK(hipMemcpyAsync(hh2, c->bH.p, (size_t)ka * s * sizeof(double2), hipMemcpyDeviceToHost, st));
            launch_bupd(st, ne, ka, s, Vg(g), LV, c->bH.p, W, S, W, S, -1.0, 1.0);
          }
          CK(cholqr2(c, s, W, c->bw1.p + g0[g], c->bw2.p + g0[g], S, Rk, ok, reorth ? nullptr : hG1,
                     Vg(g) + (int64_t)(k + 1) * s, LV));
        }
        if (!ok) {  // W lost rank: this step of the group is not used, the group restarts
          running[g] = 0;
          continue;
        }
        P.assign((size_t)(k + 2) * ss, 0.0);
        if (two_pass || reorth)
          for (size_t e = 0; e < (size_t)ka * s; ++e) P[e] = cd(hh1[e].x + hh2[e].x, hh1[e].y + hh2[e].y);
        else
          for (size_t e = 0; e < (size_t)ka * s; ++e) P[e] = cd(hh1[e].x, hh1[e].y);
        for (size_t e = 0; e < ss; ++e) P[(size_t)ka * s + e] = Rk[e];
        ls[g].add(k, P);
        kk[g] = k + 1;
        ++steps[g];
        double est = 0;
        for (int j = 0; j < s; ++j) est = std::max(est, ls[g].colres(j) / bn[g0[g] + j]);
        if (est <= rtol) running[g] = 0;
      }
      c->prof.end(K_CGS);
      ++total;
    }
    // X_g += [Z_0 .. Z_kk-1] Y_g
    for (int g = 0; g < G; ++g) {
      if (!active[g]) continue;
      if (kk[g] == 0) return set_err(MX_ENOTCONV, "block FGMRES: the first block of a cycle lost rank");
      const int s = gs[g];
      ls[g].solve(reinterpret_cast<double*>(c->hb + 2 * 32 * 32));
      MX_HIP_CHECK(hipMemcpyAsync(c->bH.p, c->hb + 2 * 32 * 32, (size_t)kk[g] * s * s * sizeof(double2),
                                  hipMemcpyHostToDevice, st));
      launch_bupd(st, ne, kk[g] * s, s, Zg(g), (int64_t)m * s, c->bH.p, c->x.p + g0[g], S, c->x.p + g0[g], S, 1.0,
                  1.0);
      CK(sync(c));  // the host buffer of Y is reused by the next group
    }
    CK(spmm(c, c->x.p, c->r.p, S));
    launch_bminus(st, blk, c->b.p, c->r.p);
    MX_HIP_CHECK(hipGetLastError());
    CK(true_residual());
    ++cycles;
  }
  auto t1 = std::chrono::steady_clock::now();
  if (info) {
    int mx_ = 0;
    for (int g = 0; g < G; ++g)
      for (int j = g0[g]; j < g0[g + 1]; ++j) {
        if (info->iters) info->iters[j] = steps[g];
        if (info->relres) info->relres[j] = rr[j];
        mx_ = std::max(mx_, steps[g]);
      }
    info->iters_max = mx_;
    info->cycles = cycles;
    info->fallback = 0;
    info->t_iter = std::chrono::duration<double>(t1 - t0).count();
    info->t_assemble = c->t_assemble;
    info->t_setup = c->t_setup;
    info->t_lu = c->t_lu;
  }
  return rc;
}

// The solver of every solve: block FGMRES when selected and applicable, else
// the pseudo-block FGMRES described with the autotuner above.
int fgmres(mx_ctx* c, int nrhs, double rtol, mx_solve_info* info, const std::function<int()>* on_cycle = nullptr) {
  bool block_fallback = false;
  const bool block_mode = c->krylov_mode != MX_KRYLOV_PSEUDO_BLOCK && !on_cycle;
  // with the learned term on, block mode first runs the pseudo-block solver
  // with the judged learned term and hands over to block FGMRES once the
  // judge has switched the term off
  bool learned_first = block_mode && c->coarse_use && c->coarse_geom && c->coarse_weights;
  if (block_mode && !learned_first) {
    const int rcb = block_fgmres(c, nrhs, rtol, info);
    if (rcb != kBlockFallback) return rcb;
    block_fallback = true;
  }
  const int m = c->ws_m;
  const int64_t ne = c->topo.ne;
  const int64_t blk = ne * (int64_t)nrhs;
  hipStream_t s = c->stream;
  auto t0 = std::chrono::steady_clock::now();
  CK(autotune(c, nrhs));
  launch_norm(s, ne, nrhs, c->b.p, c->normpart.p, c->bnorm.p);
  launch_fill_zero<double2>(s, blk, c->x.p);
  MX_HIP_CHECK(hipMemcpyAsync(c->r.p, c->b.p, blk * sizeof(double2), hipMemcpyDeviceToDevice, s));
  std::vector<double> bn(nrhs), rr(nrhs);
  MX_HIP_CHECK(hipMemcpyAsync(c->h_vec, c->bnorm.p, nrhs * sizeof(double), hipMemcpyDeviceToHost, s));
  CK(sync(c));
  for (int j = 0; j < nrhs; ++j) bn[j] = c->h_vec[j];
  std::vector<int32_t> iters(nrhs, 0);
  std::vector<char> done(nrhs, 0);
  int total = 0, cycles = 0;
  int rc = MX_OK;
  // relative residual of the current r
  auto true_residual = [&]() -> int {
    launch_norm(s, ne, nrhs, c->r.p, c->normpart.p, c->beta.p);
    MX_HIP_CHECK(hipMemcpyAsync(c->h_vec, c->beta.p, nrhs * sizeof(double), hipMemcpyDeviceToHost, s));
    CK(sync(c));
    for (int j = 0; j < nrhs; ++j) rr[j] = bn[j] > 0 ? c->h_vec[j] / bn[j] : 0.0;
    return MX_OK;
  };
  CK(true_residual());
  c->coarse_off_now = false;
  const bool coarse_on = c->coarse_use && c->coarse_geom && c->coarse_weights;
  if (coarse_on) {
    hipLaunchKernelGGL(k_zero_i32, dim3(1), dim3(64), 0, s, 1, c->cflag.p);
    CK(ensure_learned_ws(c, nrhs));
  }
  int fallback = 0;
  int judge_steps = 0;
  double judge_sum = 0;
  std::vector<double2> hj_dot(nrhs);
  std::vector<double> hj_aq(nrhs), hj_t(nrhs);
  // Gram-Schmidt (twice), normalisation and the Givens update of step k
  auto arnoldi_tail = [&](int k) -> int {
    double2* w = c->V.p + (k + 1) * blk;
    if (nrhs <= 32 && k + 1 <= cgs_fused_max()) {
      // first pass: all k+1 coefficients in one sweep; second pass fused:
      // update with h1 and form h2, then update with h2 and ||w||
      launch_cgs_pass(s, ne, nrhs, c->V.p, blk, k + 1, nullptr, w, c->dotpart.p, nullptr, c->h1.p, nullptr);
      launch_cgs_pass(s, ne, nrhs, c->V.p, blk, k + 1, c->h1.p, w, c->dotpart.p, nullptr, c->h2.p, nullptr);
      launch_cgs_pass(s, ne, nrhs, c->V.p, blk, k + 1, c->h2.p, w, nullptr, c->normpart.p, nullptr, c->hn.p);
    } else {
      launch_dot(s, ne, nrhs, c->V.p, blk, k + 1, w, c->dotpart.p, c->h1.p);
      launch_update(s, ne, nrhs, c->V.p, blk, k + 1, c->h1.p, w);
      launch_dot(s, ne, nrhs, c->V.p, blk, k + 1, w, c->dotpart.p, c->h2.p);
      launch_update(s, ne, nrhs, c->V.p, blk, k + 1, c->h2.p, w);
      launch_norm(s, ne, nrhs, w, c->normpart.p, c->hn.p);
    }
    launch_scale(s, ne, nrhs, w, c->hn.p, w);
    launch_givens(s, k, m, nrhs, c->h1.p, c->h2.p, c->hn.p, c->H.p, c->cs.p, c->sn.p, c->g.p, c->bnorm.p, rtol,
                  c->conv.p, c->kdone.p, c->res.p);
    MX_HIP_CHECK(hipGetLastError());
    return MX_OK;
  };
  // one whole step with the one-level preconditioner: kernel launches only
  auto plain_step = [&](int k) -> int {
    CK(apply_precond(c, c->V.p + k * blk, c->Z.p + k * blk, nrhs));
    CK(spmm(c, c->Z.p + k * blk, c->V.p + (k + 1) * blk, nrhs));
    c->prof.begin(K_CGS);
    CK(arnoldi_tail(k));
    c->prof.end(K_CGS);
    return MX_OK;
  };
  // Graphs are used without profiling; a step runs eagerly the first time
  // it is reached under the current buffers/sizes/tolerance and is captured
  // and replayed from the second time on.
  const bool use_graphs = c->graphs_on && !c->prof.on;
  if (use_graphs) {
    const uint64_t sig = step_signature(c, nrhs, m, rtol);
    if (sig != c->g_sig || (int)c->gexec.size() != m) {
      c->drop_graphs();
      c->g_sig = sig;
      c->gexec.assign(m, nullptr);
      c->gseen.assign(m, 0);
    }
  }
  auto graph_step = [&](int k) -> int {
    if (!c->graphs_on) return plain_step(k);
    if (!c->gexec[k]) {
      if (!c->gseen[k]) {
        c->gseen[k] = 1;
        return plain_step(k);
      }
      hipGraph_t g = nullptr;
      MX_HIP_CHECK(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
      const int rc_step = plain_step(k);
      const hipError_t e_end = hipStreamEndCapture(s, &g);
      hipError_t e_inst = hipErrorUnknown;
      if (rc_step == MX_OK && e_end == hipSuccess && g)
        e_inst = hipGraphInstantiate(&c->gexec[k], g, nullptr, nullptr, 0);
      if (g) (void)hipGraphDestroy(g);
      if (rc_step != MX_OK || e_end != hipSuccess || e_inst != hipSuccess) {
        // capture not possible here: run eagerly from now on
        (void)hipGetLastError();
        c->gexec[k] = nullptr;
        c->graphs_on = false;
        return plain_step(k);
      }
    }
    MX_HIP_CHECK(hipGraphLaunch(c->gexec[k], s));
    return MX_OK;
  };
  for (;;) {
    if (on_cycle) CK((*on_cycle)());
    std::vector<double> rr_start(rr);
    bool all = true;
    for (int j = 0; j < nrhs; ++j) {
      if (rr[j] <= rtol) done[j] = 1;
      all = all && done[j];
    }
    if (all) break;
    if (learned_first && c->coarse_off_now) {
      std::vector<int32_t> bit(nrhs, 0);
      std::vector<double> brr(nrhs, 0.0);
      mx_solve_info binfo{};
      binfo.iters = bit.data();
      binfo.relres = brr.data();
      const int rcb = block_fgmres(c, nrhs, rtol, &binfo, true);
      if (rcb != kBlockFallback) {
        for (int j = 0; j < nrhs; ++j) {
          iters[j] += bit[j];
          rr[j] = brr[j];
        }
        cycles += binfo.cycles;
        rc = rcb;
        break;
      }
      learned_first = false;  // continue with the pseudo-block solver
      block_fallback = true;
    }
    if (total >= c->maxit) {
      rc = set_err(MX_ENOTCONV, "FGMRES reached maxit=" + std::to_string(c->maxit));
      break;
    }
    // new cycle: V_0 = r / beta, g = beta e_1
    launch_scale(s, ne, nrhs, c->r.p, c->beta.p, c->V.p);
    hipLaunchKernelGGL(k_set_g0, dim3((unsigned)(((m + 1) * nrhs + 255) / 256)), dim3(256), 0, s, m, nrhs,
                       c->beta.p, c->g.p);
    hipLaunchKernelGGL(k_zero_i32, dim3((unsigned)((nrhs + 255) / 256)), dim3(256), 0, s, nrhs, c->conv.p);
    hipLaunchKernelGGL(k_zero_i32, dim3((unsigned)((nrhs + 255) / 256)), dim3(256), 0, s, nrhs, c->kdone.p);
    int ksteps = 0;
    for (int k = 0; k < m; ++k) {
      double2* vk = c->V.p + k * blk;
      double2* zk = c->Z.p + k * blk;
      double2* w = c->V.p + (k + 1) * blk;
      bool judged = false;
      if (coarse_on && !c->coarse_off_now) {
        // plain ORAS judges the learned term: z = M^{-1} v + theta q with the
        // per-transmitter theta minimising ||v - A z||
        CK(precond_learned(c, vk, zk, w, nrhs));
        judged = true;
        c->prof.begin(K_CGS);
        CK(arnoldi_tail(k));
        c->prof.end(K_CGS);
      } else if (use_graphs) {
        CK(graph_step(k));
      } else {
        CK(plain_step(k));
      }
      MX_HIP_CHECK(hipMemcpyAsync(c->h_conv, c->conv.p, nrhs * sizeof(int32_t), hipMemcpyDeviceToHost, s));
      if (coarse_on && !c->coarse_off_now)
        MX_HIP_CHECK(hipMemcpyAsync(c->h_kd, c->cflag.p, sizeof(int32_t), hipMemcpyDeviceToHost, s));
      if (judged) {
        MX_HIP_CHECK(hipMemcpyAsync(hj_dot.data(), c->thdot.p, nrhs * sizeof(double2), hipMemcpyDeviceToHost, s));
        MX_HIP_CHECK(hipMemcpyAsync(hj_aq.data(), c->thnrm.p, nrhs * sizeof(double), hipMemcpyDeviceToHost, s));
        MX_HIP_CHECK(hipMemcpyAsync(hj_t.data(), c->thtn.p, nrhs * sizeof(double), hipMemcpyDeviceToHost, s));
      }
      CK(sync(c));
      if (judged) {
        // squared reduction of the local preconditioned residual the learned
        // term brings: ||v - A(z1 + theta q)||^2 / ||v - A z1||^2
        double red = 0;
        int cnt = 0;
        for (int j = 0; j < nrhs; ++j) {
          const double d = hj_aq[j] * hj_t[j];
          if (d > 0) {
            const double a = std::hypot(hj_dot[j].x, hj_dot[j].y) / d;
            red += 1.0 - a * a;
            ++cnt;
          }
        }
        judge_sum += cnt ? red / cnt : 1.0;
        if (++judge_steps == 4 && judge_sum / judge_steps > 0.95 * 0.95) {
          // the learned term removes less than 5% of what plain ORAS leaves: drop it
          c->coarse_off_now = true;
          fallback = 3;
        }
      }
      if (coarse_on && !c->coarse_off_now && c->h_kd[0] != 0) {
        // non-finite network output: drop this cycle, continue with plain ORAS
        c->coarse_off_now = true;
        fallback = 1;
        ksteps = -1;
        break;
      }
      ksteps = k + 1;
      ++total;
      int nconv = 0;
      for (int j = 0; j < nrhs; ++j) nconv += c->h_conv[j] != 0 || done[j];
      if (nconv == nrhs || total >= c->maxit) break;
      if (learned_first && c->coarse_off_now) break;  // hand over to block FGMRES
    }
    if (ksteps < 0) {
      // the cycle is dropped with x unchanged (r still holds b - A x)
      CK(true_residual());
      continue;
    }
    launch_lsq(s, ksteps, m, nrhs, c->H.p, c->g.p, c->conv.p, c->kdone.p, c->y.p);
    launch_xupdate(s, ne, nrhs, c->Z.p, blk, c->y.p, c->kdone.p, c->x.p);
    CK(spmm(c, c->x.p, c->r.p, nrhs));
    launch_bminus(s, blk, c->b.p, c->r.p);
    MX_HIP_CHECK(hipMemcpyAsync(c->h_kd, c->kdone.p, nrhs * sizeof(int32_t), hipMemcpyDeviceToHost, s));
    CK(true_residual());
    for (int j = 0; j < nrhs; ++j)
      if (!done[j]) iters[j] += c->h_kd[j];
    ++cycles;
    if (coarse_on && !c->coarse_off_now) {
      // plain one-level Schwarz judges the learned term: a full cycle that does
      // not reduce the worst residual by 10% switches it off for this solve
      double worst = 0;
      for (int j = 0; j < nrhs; ++j)
        if (!done[j] && rr_start[j] > 0) worst = std::max(worst, rr[j] / rr_start[j]);
      if (worst > 0.9) {
        c->coarse_off_now = true;
        fallback = 2;
      }
    }
  }
  if (fallback) c->coarse_fallbacks++;
  auto t1 = std::chrono::steady_clock::now();
  if (info) {
    int mx_ = 0;
    for (int j = 0; j < nrhs; ++j) {
      if (info->iters) info->iters[j] = iters[j];
      if (info->relres) info->relres[j] = rr[j];
      mx_ = std::max(mx_, iters[j]);
    }
    info->iters_max = mx_;
    info->cycles = cycles;
    info->fallback = fallback ? fallback : (block_fallback ? 4 : 0);
    info->t_iter = std::chrono::duration<double>(t1 - t0).count();
    info->t_assemble = c->t_assemble;
    info->t_setup = c->t_setup;
    info->t_lu = c->t_lu;
  }
  return rc;
}


// host Cholesky inverse of an SPD n x n matrix (row-major, in place)
bool spd_inverse(std::vector<double>& A, int n) {
  std::vector<double> L(A.size(), 0.0);
  for (int j = 0; j < n; ++j) {
    double d = A[(size_t)j * n + j];
    for (int k = 0; k < j; ++k) d -= L[(size_t)j * n + k] * L[(size_t)j * n + k];
    if (!(d > 0)) return false;
    d = std::sqrt(d);
    L[(size_t)j * n + j] = d;
    for (int i = j + 1; i < n; ++i) {
      double v = A[(size_t)i * n + j];
      for (int k = 0; k < j; ++k) v -= L[(size_t)i * n + k] * L[(size_t)j * n + k];
      L[(size_t)i * n + j] = v / d;
    }
  }
  // inverse = L^{-T} L^{-1}: solve column by column
  std::vector<double> X((size_t)n * n, 0.0), y(n);
  for (int c = 0; c < n; ++c) {
    for (int i = 0; i < n; ++i) {
      double v = i == c ? 1.0 : 0.0;
      for (int k = 0; k < i; ++k) v -= L[(size_t)i * n + k] * y[k];
      y[i] = v / L[(size_t)i * n + i];
    }
    for (int i = n - 1; i >= 0; --i) {
      double v = y[i];
      for (int k = i + 1; k < n; ++k) v -= L[(size_t)k * n + i] * X[(size_t)k * n + c];
      X[(size_t)i * n + c] = v / L[(size_t)i * n + i];
    }
  }
  A.swap(X);
  return true;
}

// lattices, prolongations and least-squares operators of the current decomposition
// Ranges of the triangular solves from the band bookkeeping of the
// factorisation: row tile t of L has non-zeros in the column tiles
// [lo_t, t), lo_t = first panel whose L part reaches t; row tile t of U in
// (t, ext_u[t]]. Also the tile counts of the factorisation and of one
// lower + upper solve per right-hand side.
int triangular_ranges(mx_ctx* c) {
  const Decomposition& D = c->dec;
  const int np = c->band_np;
  const size_t n = (size_t)D.nsub * np;
  std::vector<int32_t> el(n), eu(n), lo(n, 0);
  int64_t work = 0;
  MX_HIP_CHECK(hipMemcpyAsync(el.data(), c->ext_l.p, n * sizeof(int32_t), hipMemcpyDeviceToHost, c->stream));
  MX_HIP_CHECK(hipMemcpyAsync(eu.data(), c->ext_u.p, n * sizeof(int32_t), hipMemcpyDeviceToHost, c->stream));
  MX_HIP_CHECK(hipMemcpyAsync(&work, c->band_work.p, sizeof(int64_t), hipMemcpyDeviceToHost, c->stream));
  CK(sync(c));
  int64_t tiles_l = 0, tiles_u = 0;
  for (int s = 0; s < D.nsub; ++s) {
    const int nt = D.Npad[s] / 64;
    const int32_t* e = el.data() + (size_t)s * np;
    int32_t* l = lo.data() + (size_t)s * np;
    for (int t = 0; t < nt; ++t) {
      int f = t;
      for (int q = 0; q < t; ++q)
        if (e[q] >= t) { f = q; break; }
      l[t] = f;
      // off-diagonal tiles of each solve plus the diagonal (inverse) tile
      tiles_l += (t - f) + 1;
      tiles_u += (std::min(eu[(size_t)s * np + t], nt - 1) - t) + 1;
    }
  }
  CK(c->trs_lo.upload(lo, c->stream));
  CK(c->trs_hi.upload(eu, c->stream));
  c->lu_tiles = work;
  c->trsm_tiles_l = tiles_l;
  c->trsm_tiles_u = tiles_u;
  return sync(c);
}

int coarse_prepare(mx_ctx* c) {
  const Topology& T = c->topo;
  const Decomposition& D = c->dec;
  const int nsub = D.nsub;
  const int64_t nrows = D.dof_ptr[nsub];
  std::vector<int32_t> rs(nrows);
  for (int i = 0; i < nsub; ++i)
    for (int64_t k = D.dof_ptr[i]; k < D.dof_ptr[i + 1]; ++k) rs[k] = i;
  std::vector<double> box(6 * (size_t)nsub);
  for (int i = 0; i < nsub; ++i) {
    double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int64_t k = D.tet_ptr[i]; k < D.tet_ptr[i + 1]; ++k)
      for (int q = 0; q < 4; ++q) {
        const double* x = &T.xyz[3 * (size_t)T.ts[4 * (size_t)D.tets[k] + q]];
        for (int d = 0; d < 3; ++d) { lo[d] = std::min(lo[d], x[d]); hi[d] = std::max(hi[d], x[d]); }
      }
    for (int d = 0; d < 3; ++d) { box[6 * i + d] = lo[d]; box[6 * i + 3 + d] = hi[d]; }
  }
  CK(c->row_sub.upload(rs, c->stream));
  CK(c->cbox.upload(box, c->stream));
  CK(c->edges_dev.upload(T.edges, c->stream));
  CK(c->cnbr_ptr.upload(D.nbr_ptr, c->stream));
  CK(c->cnbrs.upload(D.nbrs.empty() ? std::vector<int32_t>(1, 0) : D.nbrs, c->stream));
  CK(c->cP.alloc((size_t)nrows * NCO));
  CK(c->cpart.alloc((size_t)pool_scratch_floats(nsub)));
  launch_coarse_P(c->stream, nrows, c->row_sub.p, c->dofs.p, c->edges_dev.p, c->xyz.p, c->cbox.p, c->cP.p);
  CK(c->cpdp.alloc((size_t)nsub * NCO * NCO));
  DBuf<double> Dw;
  CK(Dw.upload(D.D, c->stream));
  launch_pdp(c->stream, nsub, c->dof_ptr.p, c->cP.p, Dw.p, c->cpdp.p);
  MX_HIP_CHECK(hipGetLastError());
  std::vector<double> G((size_t)nsub * NCO * NCO);
  MX_HIP_CHECK(hipMemcpyAsync(G.data(), c->cpdp.p, G.size() * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  CK(sync(c));
  bool ok = true;
#pragma omp parallel for schedule(dynamic, 1)
  for (int i = 0; i < nsub; ++i) {
    std::vector<double> A(G.begin() + (size_t)i * NCO * NCO, G.begin() + (size_t)(i + 1) * NCO * NCO);
    double tr = 0;
    for (int k = 0; k < NCO; ++k) tr += A[(size_t)k * NCO + k];
    const double lam = 1e-6 * tr / NCO;
    for (int k = 0; k < NCO; ++k) A[(size_t)k * NCO + k] += lam;
    if (!spd_inverse(A, NCO)) ok = false;
    std::copy(A.begin(), A.end(), G.begin() + (size_t)i * NCO * NCO);
  }
  if (!ok) return set_err(MX_EINVAL, "coarse least-squares matrix is not positive definite");
  CK(c->cG.upload(G, c->stream));
  CK(c->cscale.alloc(256));
  CK(c->cflag.alloc(4));
  CK(sync(c));
  c->coarse_geom = true;
  return MX_OK;
}

// ---------------------------------------------------------------------------
// waveguide ports (Sec. IV-B, eq. (1))
// ---------------------------------------------------------------------------
double2 port_beta(double k0, const mx_port& p) {
  const double2 z = make_double2(k0 * k0 * p.eps.re - (M_PI / p.a) * (M_PI / p.a), k0 * k0 * p.eps.im);
  double2 b = csqrt_host(z);  // principal root; the decaying branch has Im <= 0
  if (b.y > 0) b = make_double2(-b.x, -b.y);
  return b;
}

struct PortFrame {
  double c[3], n[3], u[3], v[3];
};
PortFrame port_frame(const mx_port& p) {
  PortFrame f;
  double nn = std::sqrt(p.normal[0] * p.normal[0] + p.normal[1] * p.normal[1] + p.normal[2] * p.normal[2]);
  for (int k = 0; k < 3; ++k) { f.c[k] = p.centre[k]; f.n[k] = p.normal[k] / nn; }
  const double un = p.u[0] * f.n[0] + p.u[1] * f.n[1] + p.u[2] * f.n[2];
  for (int k = 0; k < 3; ++k) f.u[k] = p.u[k] - un * f.n[k];
  const double uu = std::sqrt(f.u[0] * f.u[0] + f.u[1] * f.u[1] + f.u[2] * f.u[2]);
  for (int k = 0; k < 3; ++k) f.u[k] /= uu;
  f.v[0] = f.n[1] * f.u[2] - f.n[2] * f.u[1];
  f.v[1] = f.n[2] * f.u[0] - f.n[0] * f.u[2];
  f.v[2] = f.n[0] * f.u[1] - f.n[1] * f.u[0];
  return f;
}

// Face classification, metallic edges, and the port moments
// m_p[e] = int_port e_p . N_e dS, |e_p|^2 = int_port e_p . e_p dS, with the
// tangential edge functions of each face, N_ab = l_a grad l_b - l_b grad l_a,
// grad l_0 = n x (x2 - x1) / (2|F|) and cyclically, and the 7-point
// degree-5 triangle rule of Dunavant (1985).
int build_ports(mx_ctx* c) {
  const Topology& T = c->topo;
  static const int LF[4][3] = {{0, 1, 2}, {0, 1, 3}, {0, 2, 3}, {1, 2, 3}};
  static const int FE[3][2] = {{0, 1}, {0, 2}, {1, 2}};
  auto local_edge = [](int a, int b) {  // (a < b) tetrahedron vertex pair -> local edge
    static const int tab[4][4] = {{-1, 0, 1, 2}, {0, -1, 3, 4}, {1, 3, -1, 5}, {2, 4, 5, -1}};
    return tab[a][b];
  };
  static const double QA = 0.0597158717897698, QB = 0.4701420641051151;
  static const double QC = 0.7974269853530873, QD = 0.1012865073234563;
  static const double QL[7][3] = {{1.0 / 3, 1.0 / 3, 1.0 / 3}, {QA, QB, QB}, {QB, QA, QB}, {QB, QB, QA},
                                  {QC, QD, QD}, {QD, QC, QD}, {QD, QD, QC}};
  static const double QW[7] = {0.225, 0.1323941527885062, 0.1323941527885062, 0.1323941527885062,
                               0.1259391805448271, 0.1259391805448271, 0.1259391805448271};
  const int np = (int)c->ports.size();
  std::vector<PortFrame> fr(np);
  for (int p = 0; p < np; ++p) fr[p] = port_frame(c->ports[p]);
  const int64_t nbf = T.nbf;
  c->face_port.assign(nbf, -1);
  std::vector<char> pec(T.ne, 0);
  std::vector<std::vector<std::pair<int32_t, double>>> mom(np);
  c->pm_norm.assign(np, 0.0);
  for (int64_t f = 0; f < nbf; ++f) {
    const int t = T.bf_tet[f], lf = T.bf_lf[f];
    int vloc[3];
    double P[3][3];
    for (int k = 0; k < 3; ++k) {
      vloc[k] = LF[lf][k];
      const int vid = T.ts[4 * (size_t)t + vloc[k]];
      for (int d = 0; d < 3; ++d) P[k][d] = T.xyz[3 * (size_t)vid + d];
    }
    double cen[3];
    for (int d = 0; d < 3; ++d) cen[d] = (P[0][d] + P[1][d] + P[2][d]) / 3.0;
    int port = -1;
    for (int p = 0; p < np && port < 0; ++p) {
      const mx_port& q = c->ports[p];
      const double tol = 1e-6 * (q.a + q.b);
      double dn = 0, du = 0, dv = 0;
      for (int d = 0; d < 3; ++d) {
        const double x = cen[d] - fr[p].c[d];
        dn += x * fr[p].n[d];
        du += x * fr[p].u[d];
        dv += x * fr[p].v[d];
      }
      if (std::fabs(dn) <= tol && std::fabs(du) <= 0.5 * q.a + tol && std::fabs(dv) <= 0.5 * q.b + tol) port = p;
    }
    c->face_port[f] = port;
    int32_t ge[3];
    for (int k = 0; k < 3; ++k) ge[k] = T.t2e[6 * (size_t)t + local_edge(vloc[FE[k][0]], vloc[FE[k][1]])];
    if (port < 0) {
      if (c->pec_walls)
        for (int k = 0; k < 3; ++k) pec[ge[k]] = 1;
      continue;
    }
    // face geometry
    double e01[3], e02[3], nrm[3];
    for (int d = 0; d < 3; ++d) { e01[d] = P[1][d] - P[0][d]; e02[d] = P[2][d] - P[0][d]; }
    nrm[0] = e01[1] * e02[2] - e01[2] * e02[1];
    nrm[1] = e01[2] * e02[0] - e01[0] * e02[2];
    nrm[2] = e01[0] * e02[1] - e01[1] * e02[0];
    const double twoA = std::sqrt(nrm[0] * nrm[0] + nrm[1] * nrm[1] + nrm[2] * nrm[2]);
    for (int d = 0; d < 3; ++d) nrm[d] /= twoA;
    double gl[3][3];
    for (int k = 0; k < 3; ++k) {
      const double* xa = P[(k + 1) % 3];
      const double* xb = P[(k + 2) % 3];
      const double w[3] = {xb[0] - xa[0], xb[1] - xa[1], xb[2] - xa[2]};
      gl[k][0] = (nrm[1] * w[2] - nrm[2] * w[1]) / twoA;
      gl[k][1] = (nrm[2] * w[0] - nrm[0] * w[2]) / twoA;
      gl[k][2] = (nrm[0] * w[1] - nrm[1] * w[0]) / twoA;
    }
    const mx_port& q = c->ports[port];
    double acc[3] = {0, 0, 0};
    for (int iq = 0; iq < 7; ++iq) {
      double x[3];
      for (int d = 0; d < 3; ++d) x[d] = QL[iq][0] * P[0][d] + QL[iq][1] * P[1][d] + QL[iq][2] * P[2][d];
      double su = 0;
      for (int d = 0; d < 3; ++d) su += (x[d] - fr[port].c[d]) * fr[port].u[d];
      const double amp = std::sin(M_PI * (su + 0.5 * q.a) / q.a);
      const double wq = QW[iq] * 0.5 * twoA;
      c->pm_norm[port] += wq * amp * amp;
      for (int k = 0; k < 3; ++k) {
        const int a = FE[k][0], b = FE[k][1];
        double Nv = 0;  // e . N_k with e = amp v
        for (int d = 0; d < 3; ++d) Nv += fr[port].v[d] * (QL[iq][a] * gl[b][d] - QL[iq][b] * gl[a][d]);
        acc[k] += wq * amp * Nv;
      }
    }
    for (int k = 0; k < 3; ++k) mom[port].push_back({ge[k], acc[k]});
  }
  c->pec_list.clear();
  for (int64_t e = 0; e < T.ne; ++e)
    if (pec[e]) c->pec_list.push_back((int32_t)e);
  // sum the moments per (port, edge), metallic edges excluded
  c->pm_ptr.assign(1, 0);
  c->pm_edge.clear();
  c->pm_val.clear();
  for (int p = 0; p < np; ++p) {
    if (c->pm_norm[p] <= 0) return set_err(MX_EINVAL, "port " + std::to_string(p) + " covers no boundary face");
    auto& m = mom[p];
    std::stable_sort(m.begin(), m.end(), [](const std::pair<int32_t, double>& x, const std::pair<int32_t, double>& y) {
      return x.first < y.first;
    });
    for (size_t i = 0; i < m.size();) {
      size_t j = i;
      double sum = 0;
      while (j < m.size() && m[j].first == m[i].first) sum += m[j++].second;
      if (!pec[m[i].first]) {
        c->pm_edge.push_back(m[i].first);
        c->pm_val.push_back(sum);
      }
      i = j;
    }
    c->pm_ptr.push_back((int64_t)c->pm_edge.size());
  }
  std::vector<int32_t> flag(T.ne, 0);
  for (int32_t e : c->pec_list) flag[e] = 1;
  CK(c->pec_flag.upload(flag, c->stream));
  CK(c->pec_rows.upload(c->pec_list, c->stream));
  c->pec_local_ready = false;
  return MX_OK;
}

bool pec_active(const mx_ctx* c) { return !c->ports.empty() && !c->pec_list.empty(); }

int fill_pool(mx_ctx* c) {
  const Topology& T = c->topo;
  const size_t need = 36 * (size_t)T.nt + 9 * (size_t)T.nbf + (c->have_dec ? 9 * c->dec.if_tet.size() : 0);
  CK(c->pool.alloc(need));
  launch_element(c->stream, T.nt, c->ts.p, c->xyz.p, c->eps.p, c->eps_kind, c->k0 * c->k0, c->pool.p);
  const double2* kface = nullptr;
  if (!c->ports.empty()) {
    // port faces j beta_p, metallic faces nothing (their edges are
    // eliminated), other faces the impedance j k_b
    std::vector<double2> kf(T.nbf);
    std::vector<double2> beta(c->ports.size());
    for (size_t p = 0; p < c->ports.size(); ++p) beta[p] = port_beta(c->k0, c->ports[p]);
    for (int64_t f = 0; f < T.nbf; ++f) {
      const int p = c->face_port[f];
      kf[f] = p >= 0 ? beta[p] : (c->pec_walls ? make_double2(0.0, 0.0) : c->kb);
    }
    CK(c->face_k.upload(kf, c->stream));
    kface = c->face_k.p;
  }
  launch_face(c->stream, (int32_t)T.nbf, c->bf_tet.p, c->bf_lf.p, c->ts.p, c->xyz.p, c->eps.p, c->eps_kind, 0,
              c->k0, c->kb, c->pool.p + 36 * (size_t)T.nt, kface);
  if (c->have_dec && !c->dec.if_tet.empty())
    launch_face(c->stream, (int32_t)c->dec.if_tet.size(), c->if_tet.p, c->if_lf.p, c->ts.p, c->xyz.p, c->eps.p,
                c->eps_kind, 1, c->k0, c->kb, c->pool.p + 36 * (size_t)T.nt + 9 * (size_t)T.nbf);
  MX_HIP_CHECK(hipGetLastError());
  c->pool_filled = need;
  return MX_OK;
}

int build_sources(mx_ctx* c, const mx_sources* src, SourceSet& out) {
  if (!src || src->n <= 0 || !src->pos || !src->moment) return set_err(MX_EINVAL, "empty source set");
  if (out.same(src)) return MX_OK;
  out.pos.assign(src->pos, src->pos + 3 * (size_t)src->n);
  out.mom.assign((const double*)src->moment, (const double*)src->moment + 6 * (size_t)src->n);
  out.ptr.assign(1, 0);
  out.edge.clear();
  out.val.clear();
  std::vector<int32_t> e;
  std::vector<double> v;
  for (int j = 0; j < src->n; ++j) {
    double pr[3], pi[3];
    for (int d = 0; d < 3; ++d) {
      pr[d] = src->moment[3 * j + d].re;
      pi[d] = src->moment[3 * j + d].im;
    }
    if (!point_functional(c->topo, &src->pos[3 * (size_t)j], pr, pi, e, v)) {
      out.pos.clear();
      return set_err(MX_EINVAL, "source/receiver " + std::to_string(j) + " lies outside the mesh");
    }
    for (size_t k = 0; k < e.size(); ++k) {
      out.edge.push_back(e[k]);
      out.val.push_back(make_double2(v[2 * k], v[2 * k + 1]));
    }
    out.ptr.push_back((int64_t)out.edge.size());
  }
  return MX_OK;
}

}  // namespace

// Workgroup order of the triangular solves: one workgroup per subdomain and
// 32 right-hand sides, all resident at once when there are at most two per
// compute unit. Workgroups b and b + nsub/2 are then dealt to the same compute
// unit, so the b-th largest subdomain is paired with the b-th smallest and the
// per-unit work is even; beyond that the largest subdomains go first.
static std::vector<int32_t> trsm_dispatch_order(const std::vector<int32_t>& by_size_desc) {
  const int n = (int)by_size_desc.size();
  if (n > 512) return by_size_desc;
  std::vector<int32_t> o(n);
  const int half = (n + 1) / 2;
  for (int b = 0; b < n; ++b) o[b] = b < half ? by_size_desc[b] : by_size_desc[n - 1 - (b - half)];
  return o;
}

extern "C" {

const char* mx_last_error(void) { return g_err.c_str(); }

int mx_create(mx_ctx** out, int device, void* hip_stream) {
  if (!out) return set_err(MX_EINVAL, "out is NULL");
  *out = nullptr;
  int ndev = 0;
  MX_HIP_CHECK(hipGetDeviceCount(&ndev));
  if (device < 0 || device >= ndev) return set_err(MX_EINVAL, "no such HIP device");
  mx_ctx* c = new mx_ctx();
  c->device = device;
  hipError_t e = hipSetDevice(device);
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&c->own_stream, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipEventCreate(&c->ev_lu[0]);
  if (e == hipSuccess) e = hipEventCreate(&c->ev_lu[1]);
  c->stream = hip_stream ? (hipStream_t)hip_stream : c->own_stream;
  c->prof.stream = &c->stream;
  if (e == hipSuccess) {
    const int rc = scratch_address(device, &c->scratch_dev);
    if (rc != MX_OK) {
      for (hipEvent_t ev : c->ev_lu)
        if (ev) (void)hipEventDestroy(ev);
      if (c->own_stream) (void)hipStreamDestroy(c->own_stream);
      delete c;
      return rc;
    }
  }
  if (e != hipSuccess) {
    for (hipEvent_t ev : c->ev_lu)
      if (ev) (void)hipEventDestroy(ev);
    if (c->own_stream) (void)hipStreamDestroy(c->own_stream);
    delete c;
    return hip_fail(e, "hipStreamCreate", __FILE__, __LINE__);
  }
  *out = c;
  return MX_OK;
}

int mx_destroy(mx_ctx* c) {
  if (!c) return MX_OK;
  (void)hipSetDevice(c->device);
  if (c->stream) (void)hipStreamSynchronize(c->stream);
  if (c->h_conv) (void)hipHostFree(c->h_conv);
  if (c->h_vec) (void)hipHostFree(c->h_vec);
  if (c->h_kd) (void)hipHostFree(c->h_kd);
  if (c->hb) (void)hipHostFree(c->hb);
  c->drop_graphs();
  c->prof.reset();
  for (hipEvent_t ev : c->ev_lu)
    if (ev) (void)hipEventDestroy(ev);
  if (c->own_stream) (void)hipStreamDestroy(c->own_stream);
  delete c;
  return MX_OK;
}

int mx_set_stream(mx_ctx* c, void* hip_stream) {
  if (!c) return set_err(MX_EINVAL, "NULL context");
  CK(use_device(c));
  CK(sync(c));
  c->stream = hip_stream ? (hipStream_t)hip_stream : c->own_stream;
  return MX_OK;
}

int mx_set_autotune(mx_ctx* c, int enable) {
  if (!c) return set_err(MX_EINVAL, "NULL context");
  c->autotune_on = enable != 0;
  c->lu_autotune = true;
  if (!c->autotune_on) {
    c->tune_key = 0;
    c->tune_spmm = 0;
    c->tune_trsm_paired = 1;
    c->tune_trsm_cols = 32;
    c->tune_lu_key = 0;
    c->tune_lu_group = kLuGroupDefault;
    c->lu_tuned.clear();
    c->solve_tuned.clear();
  }
  return MX_OK;
}

int mx_set_lu_group(mx_ctx* c, int32_t group) {
  if (!c) return set_err(MX_EINVAL, "NULL context");
  if (group < 0 || group > 16) return set_err(MX_EINVAL, "panel group: 1..16, or 0 for the autotuner");
  c->tune_lu_key = 0;
  c->lu_tuned.clear();
  c->lu_autotune = group == 0;
  c->tune_lu_group = group == 0 ? kLuGroupDefault : group;
  return MX_OK;
}

int mx_set_tuning(mx_ctx* c, int32_t spmm_variant, int32_t trsm_paired, int32_t trsm_cols) {
  if (!c) return set_err(MX_EINVAL, "NULL context");
  if (spmm_variant < 0 || spmm_variant > 2 || (trsm_paired != 0 && trsm_paired != 1) ||
      (trsm_cols != 16 && trsm_cols != 32))
    return set_err(MX_EINVAL, "variants: spmm 0/1/2, trsm order 0/1, trsm columns 16/32");
  if (spmm_variant == 2 && !c->win_ok)
    return set_err(MX_EINVAL, "spmm variant 2 needs an assembled mesh whose rows fit a column window");
  c->autotune_on = false;
  c->tune_key = 0;
  c->tune_spmm = spmm_variant;
  c->tune_trsm_paired = trsm_paired;
  c->tune_trsm_cols = trsm_cols;
  return MX_OK;
}

int mx_get_tuning(mx_ctx* c, mx_tuning* out) {
  if (!c || !out) return set_err(MX_EINVAL, "NULL argument");
  out->spmm_variant = c->tune_spmm;
  out->trsm_paired = c->tune_trsm_paired;
  out->trsm_cols = c->tune_trsm_cols;
  for (int i = 0; i < 3; ++i) out->spmm_ms[i] = c->tune_spmm_ms[i];
  for (int i = 0; i < 4; ++i) out->trsm_ms[i] = c->tune_trsm_ms[i];
  out->lu_group = c->tune_lu_group;
  for (int i = 0; i < 4; ++i) out->lu_ms[i] = c->tune_lu_ms[i];
  out->from_cache = (c->tune_from_cache ? 1 : 0) | (c->tune_lu_from_cache ? 2 : 0);
  return MX_OK;
}

int mx_set_graphs(mx_ctx* c, int enable) {
  if (!c) return set_err(MX_EINVAL, "NULL context");
  CK(use_device(c));
  CK(sync(c));
  c->drop_graphs();
  c->graphs_on = enable != 0;
  return MX_OK;
}

int mx_set_profiling(mx_ctx* c, int enable) {
  if (!c) return set_err(MX_EINVAL, "NULL context");
  CK(use_device(c));
  CK(sync(c));
  c->prof.reset();
  c->prof.on = enable != 0;
  return MX_OK;
}

int mx_get_kernel_times(mx_ctx* c, mx_kernel_times* out) {
  if (!c || !out) return set_err(MX_EINVAL, "NULL argument");
  CK(use_device(c));
  CK(sync(c));
  c->prof.resolve();
  std::memset(out, 0, sizeof(*out));
  for (int i = 0; i < K_NCLASS && i < MX_K_NCLASS; ++i) {
    out->ms[i] = c->prof.ms[i];
    out->launches[i] = c->prof.n[i];
  }
  return MX_OK;
}

int mx_assemble(mx_ctx* c, const mx_mesh* mesh, const mx_c128* eps, int eps_kind, double freq_hz, mx_c128 eps_b) {
  if (!c || !eps) return set_err(MX_EINVAL, "NULL argument");
  if (eps_kind != MX_EPS_P0 && eps_kind != MX_EPS_P1) return set_err(MX_EINVAL, "bad eps_kind");
  if (!(freq_hz > 0) || !std::isfinite(freq_hz)) return set_err(MX_EINVAL, "frequency must be positive");
  if (!std::isfinite(eps_b.re) || !std::isfinite(eps_b.im)) return set_err(MX_EINVAL, "non-finite eps_b");
  CK(use_device(c));
  const auto t_start = std::chrono::steady_clock::now();
  if (mesh) {
    Topology T;
    std::string err = build_topology(mesh->nv, mesh->nt, mesh->xyz, mesh->tet, T);
    if (!err.empty()) return set_err(MX_EINVAL, err);
    c->topo = std::move(T);
    c->have_mesh = true;
    c->have_dec = false;
    c->t2e.release();
    c->v2t.release();
    c->v2t_ptr.release();
    c->local_ready = c->factored = false;
    c->tx = SourceSet();
    c->rx = SourceSet();
    c->ws_nrhs = 0;
    c->ports.clear();
    c->pec_list.clear();
    c->face_port.clear();
    const Topology& t = c->topo;
    CK(c->xyz.upload(t.xyz, c->stream));
    CK(c->ts.upload(t.ts, c->stream));
    CK(c->col.upload(t.col, c->stream));
    CK(c->row_ptr.upload(t.row_ptr, c->stream));
    CK(c->cptr.upload(t.cptr, c->stream));
    c->win_ok = build_col_windows(t, kSpmmWinCap, kSpmmWinRows, c->win);
    if (c->win_ok) {
      CK(c->win_row.upload(c->win.row, c->stream));
      CK(c->win_cp.upload(c->win.cptr, c->stream));
      CK(c->win_ucol.upload(c->win.ucol, c->stream));
      CK(c->win_lcol.upload(c->win.lcol, c->stream));
    }
    CK(c->csrc.upload(t.csrc, c->stream));
    CK(c->bf_tet.upload(t.bf_tet, c->stream));
    CK(c->bf_lf.upload(t.bf_lf, c->stream));
    CK(c->val.alloc(t.nnz));
  } else if (!c->have_mesh) {
    return set_err(MX_ESTATE, "mesh is NULL and no mesh was given before");
  }
  const Topology& T = c->topo;
  const int64_t ne_eps = eps_kind == MX_EPS_P0 ? T.nt : T.nv;
  CK(c->eps.alloc(ne_eps));
  CK(copy_in(c, c->eps.p, eps, ne_eps * sizeof(double2)));
  CK(c->flag.alloc(4));
  hipLaunchKernelGGL(k_zero_i32, dim3(1), dim3(64), 0, c->stream, 1, c->flag.p);
  hipLaunchKernelGGL(k_check_finite, dim3((unsigned)((ne_eps + 255) / 256)), dim3(256), 0, c->stream, ne_eps,
                     c->eps.p, c->flag.p);
  int32_t hflag = 0;
  MX_HIP_CHECK(hipMemcpyAsync(&hflag, c->flag.p, sizeof(int32_t), hipMemcpyDeviceToHost, c->stream));
  CK(sync(c));
  if (hflag) return set_err(MX_EINVAL, "non-finite permittivity");
  c->eps_kind = eps_kind;
  c->freq = freq_hz;
  c->k0 = 2.0 * M_PI * freq_hz / C0;
  c->omega_mu0 = 2.0 * M_PI * freq_hz * MU0;
  double2 sq = csqrt_host(make_double2(eps_b.re, eps_b.im));
  c->kb = make_double2(c->k0 * sq.x, c->k0 * sq.y);
  c->prof.begin(K_ASSEMBLE);
  CK(fill_pool(c));
  launch_gather_csr(c->stream, T.nnz, c->cptr.p, c->csrc.p, c->pool.p, c->val.p);
  if (pec_active(c)) launch_pec_csr(c->stream, T.ne, c->row_ptr.p, c->col.p, c->pec_flag.p, c->val.p);
  c->prof.end(K_ASSEMBLE);
  MX_HIP_CHECK(hipGetLastError());
  CK(sync(c));
  c->assembled = true;
  c->local_ready = c->factored = false;
  c->have_forward = false;
  c->t_assemble = std::chrono::duration<double>(std::chrono::steady_clock::now() - t_start).count();
  return MX_OK;
}

// local ORAS matrices of this permittivity gathered into the factor pool
// (the precision of c->precision); tm: per-kernel profiler or NULL
int build_local(mx_ctx* c, KTimer* tm) {
  const Decomposition& D = c->dec;
  const size_t nent = (size_t)D.mat_off[D.nsub];
  const int64_t nloc = (int64_t)D.ldest.size();
  if (tm) tm->begin(K_LOCAL);
  const bool c64 = c->precision == MX_PREC_C64;
  // after a completed factorisation only the tiles inside its recorded
  // extents can be non-zero: clearing those suffices (a fraction of the bytes)
  const bool envelope = c->pool_envelope;
  c->pool_envelope = false;
  if (c64) {
    float2* F = (float2*)c->factors.p;
    if (envelope)
      launch_clear_envelope<float2>(c->stream, D.nsub, c->band_np, c->Npad.p, c->mat_off.p, c->ext_l.p, c->ext_u.p, F);
    else
      launch_fill_zero<float2>(c->stream, nent, F);
    launch_gather_dense<float2>(c->stream, nloc, c->ldest.p, c->lptr.p, c->lsrc.p, c->pool.p, F);
    launch_pad_identity<float2>(c->stream, D.nsub, c->dof_ptr.p, c->Npad.p, c->mat_off.p, F);
  } else {
    double2* F = (double2*)c->factors.p;
    if (envelope)
      launch_clear_envelope<double2>(c->stream, D.nsub, c->band_np, c->Npad.p, c->mat_off.p, c->ext_l.p, c->ext_u.p,
                                     F);
    else
      launch_fill_zero<double2>(c->stream, nent, F);
    launch_gather_dense<double2>(c->stream, nloc, c->ldest.p, c->lptr.p, c->lsrc.p, c->pool.p, F);
    launch_pad_identity<double2>(c->stream, D.nsub, c->dof_ptr.p, c->Npad.p, c->mat_off.p, F);
  }
  if (pec_active(c)) {
    if (!c->pec_local_ready) {
      // local indices of metallic edges per subdomain
      std::vector<char> pec(c->topo.ne, 0);
      for (int32_t e : c->pec_list) pec[e] = 1;
      std::vector<int64_t> ptr(1, 0);
      std::vector<int32_t> idx;
      for (int sd = 0; sd < D.nsub; ++sd) {
        for (int64_t r = D.dof_ptr[sd]; r < D.dof_ptr[sd + 1]; ++r)
          if (pec[D.dofs[r]]) idx.push_back(D.lpos[r]);
        ptr.push_back((int64_t)idx.size());
      }
      CK(c->pl_ptr.upload(ptr, c->stream));
      CK(c->pl_idx.upload(idx.empty() ? std::vector<int32_t>(1, 0) : idx, c->stream));
      c->pec_local_ready = true;
    }
    if (c64)
      launch_pec_local<float2>(c->stream, D.nsub, c->Npad.p, c->mat_off.p, c->pl_ptr.p, c->pl_idx.p,
                               (float2*)c->factors.p);
    else
      launch_pec_local<double2>(c->stream, D.nsub, c->Npad.p, c->mat_off.p, c->pl_ptr.p, c->pl_idx.p,
                                (double2*)c->factors.p);
  }
  if (tm) tm->end(K_LOCAL);
  MX_HIP_CHECK(hipGetLastError());
  return MX_OK;
}

// one banded factorisation (and the row permutation of the restriction) of
// the local matrices in the pool with `group` panels per trailing-update
// pass; ms: its device time; tm: per-kernel profiler or NULL
int factor_once(mx_ctx* c, int group, const std::vector<int32_t>& panel_rows, KTimer* tm, float* ms) {
  const Decomposition& D = c->dec;
  hipLaunchKernelGGL(k_zero_i32, dim3((unsigned)((D.nsub + 255) / 256)), dim3(256), 0, c->stream, D.nsub,
                     c->status.p);
  MX_HIP_CHECK(hipEventRecord(c->ev_lu[0], c->stream));
  const LuBand band{c->ext_l.p, c->ext_u.p, c->tptr.p, c->tbox.p, c->band_work.p, c->band0.p, c->band_lim.p,
                    c->band_np};
  if (c->precision == MX_PREC_C64)
    launch_lu<float>(c->stream, (float2*)c->factors.p, c->mat_off.p, c->Npad.p, c->order.p, c->piv.p, c->vec_off.p,
                     c->status.p, c->pswap.p, c->Nsorted, band, panel_rows, group, tm);
  else
    launch_lu<double>(c->stream, (double2*)c->factors.p, c->mat_off.p, c->Npad.p, c->order.p, c->piv.p,
                      c->vec_off.p, c->status.p, c->pswap.p, c->Nsorted, band, panel_rows, group, tm);
  if (tm) tm->begin(K_LU_INV);
  launch_perm(c->stream, D.nsub, c->Npad.p, c->vec_off.p, c->dense_edge.p, c->piv.p, c->perm.p, c->rowsrc.p);
  if (tm) tm->end(K_LU_INV);
  MX_HIP_CHECK(hipEventRecord(c->ev_lu[1], c->stream));
  MX_HIP_CHECK(hipGetLastError());
  std::vector<int32_t> st(D.nsub);
  MX_HIP_CHECK(hipMemcpyAsync(st.data(), c->status.p, D.nsub * sizeof(int32_t), hipMemcpyDeviceToHost, c->stream));
  CK(sync(c));
  for (int i = 0; i < D.nsub; ++i) {
    if (st[i] < 0)
      return set_err(MX_EHIP, "factorisation of subdomain " + std::to_string(i) + ": rows beyond the structural "
                              "band bound at column " + std::to_string(-st[i] - 1));
    if (st[i] != 0)
      return set_err(MX_EPIVOT, "zero pivot in subdomain " + std::to_string(i) + " at column " +
                                    std::to_string(st[i] - 1));
  }
  MX_HIP_CHECK(hipEventElapsedTime(ms, c->ev_lu[0], c->ev_lu[1]));
  c->pool_envelope = true;
  return MX_OK;
}

// Factorisation autotuner: at the first set-up of a shape bucket (precision,
// subdomain count, largest subdomain / 4096 unknowns) every candidate panel
// group is timed on a whole factorisation of this problem's own local
// matrices and the fastest is kept (and stored in the tuning cache under the
// bucket's key, or taken from it). *tuned: the candidates ran, so the pool
// holds factors and the caller rebuilds the local matrices.
int autotune_lu(mx_ctx* c, const std::vector<int32_t>& panel_rows, bool* tuned) {
  *tuned = false;
  if (!c->autotune_on || !c->lu_autotune) return MX_OK;
  const int nmax = c->Nsorted.empty() ? 0 : c->Nsorted[0];
  const uint64_t key = ((uint64_t)(c->precision + 1) << 48) | ((uint64_t)c->dec.nsub << 16) | (uint64_t)(nmax >> 12);
  if (key == c->tune_lu_key) return MX_OK;
  const auto seen = c->lu_tuned.find(key);
  if (seen != c->lu_tuned.end()) {
    c->tune_lu_group = seen->second;
    c->tune_lu_key = key;
    return MX_OK;
  }
  const std::string ckey = "lu:" + std::to_string(c->precision) + ":" + std::to_string(c->dec.nsub) + ":" +
                           std::to_string(nmax >> 12);
  TuneFields tf;
  if (tune_cache_get(ckey, tf) && tf.count("group") && tf["group"] >= 1 && tf["group"] <= 16) {
    c->tune_lu_group = (int)tf["group"];
    for (double& t : c->tune_lu_ms) t = 0;
    c->tune_lu_from_cache = true;
    c->tune_lu_key = key;
    c->lu_tuned[key] = c->tune_lu_group;
    return MX_OK;
  }
  int best = 0;
  for (int i = 0; i < 4; ++i) {
    if (i > 0) CK(build_local(c, nullptr));
    float ms = 0;
    *tuned = true;
    CK(factor_once(c, kLuGroups[i], panel_rows, nullptr, &ms));
    c->tune_lu_ms[i] = ms;
    if (ms < c->tune_lu_ms[best]) best = i;
  }
  c->tune_lu_group = kLuGroups[best];
  c->tune_lu_from_cache = false;
  c->tune_lu_key = key;
  c->lu_tuned[key] = c->tune_lu_group;
  tune_cache_put(ckey, {{"group", c->tune_lu_group}});
  return MX_OK;
}

int mx_setup_schwarz(mx_ctx* c, int32_t nsub, int32_t overlap, const mx_schwarz_opts* opts) {
  if (!c) return set_err(MX_EINVAL, "NULL context");
  if (!c->assembled) return set_err(MX_ESTATE, "mx_assemble must come first");
  mx_schwarz_opts o = {MX_PREC_C128, 15, 2000, 1, 0};
  if (opts) o = *opts;
  if (o.precision != MX_PREC_C128 && o.precision != MX_PREC_C64) return set_err(MX_EINVAL, "bad precision");
  CK(use_device(c));
  const auto t_start = std::chrono::steady_clock::now();
  c->restart = o.restart > 0 ? o.restart : 15;
  c->maxit = o.maxit > 0 ? o.maxit : 2000;
  if (!c->have_dec || c->dec.nsub != nsub || c->dec.overlap != overlap) {
    Decomposition D;
    std::string err = build_decomposition(c->topo, nsub, overlap, 64, D);
    if (!err.empty()) return set_err(MX_EINVAL, err);
    for (int i = 0; i < nsub; ++i)
      if (D.Npad[i] > 8192)
        return set_err(MX_EINVAL, "subdomain " + std::to_string(i) + " has more than 8192 unknowns; use more subdomains");
    c->dec = std::move(D);
    const Decomposition& d = c->dec;
    CK(c->dofs.upload(d.dofs, c->stream));
    CK(c->dof_ptr.upload(d.dof_ptr, c->stream));
    CK(c->Npad.upload(d.Npad, c->stream));
    CK(c->mat_off.upload(d.mat_off, c->stream));
    CK(c->vec_off.upload(d.vec_off, c->stream));
    CK(c->if_tet.upload(d.if_tet, c->stream));
    CK(c->if_lf.upload(d.if_lf, c->stream));
    CK(c->ldest.upload(d.ldest, c->stream));
    CK(c->lptr.upload(d.lptr, c->stream));
    CK(c->lsrc.upload(d.lsrc, c->stream));
    CK(c->pg_ptr.upload(d.pg_ptr, c->stream));
    CK(c->pg_row.upload(d.pg_row, c->stream));
    CK(c->pg_w.upload(d.pg_w, c->stream));
    CK(c->lpos.upload(d.lpos, c->stream));
    CK(c->dense_edge.upload(d.dense_edge, c->stream));
    std::vector<int32_t> ord(nsub);
    for (int i = 0; i < nsub; ++i) ord[i] = i;
    std::stable_sort(ord.begin(), ord.end(), [&](int a, int b) { return d.Npad[a] > d.Npad[b]; });
    c->Nsorted.resize(nsub);
    for (int i = 0; i < nsub; ++i) c->Nsorted[i] = d.Npad[ord[i]];
    CK(c->order.upload(ord, c->stream));
    CK(c->trsm_order.upload(trsm_dispatch_order(ord), c->stream));
    CK(c->piv.alloc(d.vec_off[nsub]));
    CK(c->perm.alloc(d.vec_off[nsub]));
    CK(c->rowsrc.alloc(d.vec_off[nsub]));
    CK(c->status.alloc(nsub));
    CK(c->pswap.alloc((size_t)nsub * (2 * lu_max_swap_rows() + 1)));
    c->band_np = d.band_np;
    CK(c->band0.upload(d.band0, c->stream));
    CK(c->band_lim.alloc((size_t)3 * nsub));
    CK(c->ext_l.alloc((size_t)nsub * c->band_np));
    CK(c->ext_u.alloc((size_t)nsub * c->band_np));
    CK(c->trs_lo.alloc((size_t)nsub * c->band_np));
    CK(c->trs_hi.alloc((size_t)nsub * c->band_np));
    CK(c->tptr.alloc((size_t)nsub + 1));
    CK(c->tbox.alloc((size_t)2 * nsub));
    CK(c->band_work.alloc(1));
    c->have_dec = true;
    c->pec_local_ready = false;
    c->pool_envelope = false;
    c->ws_nrhs = 0;
    c->coarse_geom = false;
    c->ds_graphs = 0;
  }
  const Decomposition& D = c->dec;
  c->local_ready = c->factored = false;
  c->have_forward = false;
  CK(fill_pool(c));  // interface-face blocks for this permittivity
  const size_t nent = (size_t)D.mat_off[D.nsub];
  if (c->precision != o.precision) {
    c->factors.release();
    c->pool_envelope = false;
  }
  c->precision = o.precision;
  const void* const pool_before = c->factors.p;
  CK(c->factors.alloc(nent * elem_bytes(o.precision)));
  if (c->factors.p != pool_before) c->pool_envelope = false;
  CK(build_local(c, &c->prof));
  c->local_ready = true;
  if (o.factor) {
    // rows a panel can touch: up to the last structural row tile of its own
    // and all earlier columns (partial pivoting keeps L inside that bound)
    std::vector<int32_t> panel_rows(c->band_np, 0);
    for (int i = 0; i < D.nsub; ++i) {
      const int nt = D.Npad[i] / 64;
      int hi = -1;
      for (int p = 0; p < nt; ++p) {
        hi = std::max(hi, D.band0[(size_t)i * c->band_np + p]);
        panel_rows[p] = std::max(panel_rows[p], 64 * (std::min(hi, nt - 1) + 1 - p));
      }
    }
    bool tuned = false;
    CK(autotune_lu(c, panel_rows, &tuned));
    if (tuned) CK(build_local(c, nullptr));  // the candidates' factorisations consumed the local matrices
    float lu_ms = 0;
    CK(factor_once(c, c->tune_lu_group, panel_rows, &c->prof, &lu_ms));
    c->t_lu = 1e-3 * lu_ms;
    CK(triangular_ranges(c));
    c->factored = true;
  } else {
    c->t_lu = 0;
  }
  c->coarse_use = o.coarse != 0;
  if (c->coarse_use && !c->coarse_geom) CK(coarse_prepare(c));
  CK(sync(c));
  c->t_setup = std::chrono::duration<double>(std::chrono::steady_clock::now() - t_start).count();
  return MX_OK;
}

int mx_solve_rhs(mx_ctx* c, const mx_c128* b, int32_t nrhs, double rtol, mx_c128* x, mx_solve_info* info) {
  if (!c || !b || nrhs <= 0) return set_err(MX_EINVAL, "bad arguments");
  if (!(rtol > 0)) return set_err(MX_EINVAL, "rtol must be positive");
  if (!c->factored) return set_err(MX_ESTATE, "mx_setup_schwarz (with factor=1) must come first");
  CK(use_device(c));
  CK(ensure_workspace(c, nrhs, c->restart));
  const size_t bytes = (size_t)c->topo.ne * nrhs * sizeof(double2);
  CK(copy_in(c, c->b.p, b, bytes));
  int rc = fgmres(c, nrhs, rtol, info);
  if (rc != MX_OK && rc != MX_ENOTCONV) return rc;
  CK(copy_out(c, x, c->x.p, bytes));
  CK(sync(c));
  if (rc == MX_ENOTCONV) g_err = "FGMRES reached maxit";
  return rc;
}

int mx_solve(mx_ctx* c, const mx_sources* tx, const mx_sources* rx, double rtol, mx_c128* E, mx_c128* S,
             mx_solve_info* info) {
  if (!c || !tx) return set_err(MX_EINVAL, "bad arguments");
  if (tx->n <= 0 || (rx && rx->n <= 0)) return set_err(MX_EINVAL, "empty source set");
  if (tx->n > 256) return set_err(MX_EINVAL, "at most 256 transmitters per solve");
  if (!(rtol > 0)) return set_err(MX_EINVAL, "rtol must be positive");
  if (!c->factored) return set_err(MX_ESTATE, "mx_setup_schwarz (with factor=1) must come first");
  CK(use_device(c));
  const int ntx = tx->n;
  if (!c->tx.same(tx)) {
    CK(build_sources(c, tx, c->tx));
    std::vector<int32_t> colv(c->tx.edge.size());
    for (int j = 0; j < ntx; ++j)
      for (int64_t k = c->tx.ptr[j]; k < c->tx.ptr[j + 1]; ++k) colv[k] = j;
    CK(c->s_edge.upload(c->tx.edge, c->stream));
    CK(c->s_col.upload(colv, c->stream));
    CK(c->s_val.upload(c->tx.val, c->stream));
  }
  const mx_sources* rxs = rx ? rx : tx;
  if (!c->rx.same(rxs)) {
    CK(build_sources(c, rxs, c->rx));
    CK(c->r_edge.upload(c->rx.edge, c->stream));
    CK(c->r_val.upload(c->rx.val, c->stream));
    CK(c->r_ptr.upload(c->rx.ptr, c->stream));
  }
  CK(ensure_workspace(c, ntx, c->restart));
  const int64_t blk = c->topo.ne * (int64_t)ntx;
  launch_fill_zero<double2>(c->stream, blk, c->b.p);
  launch_scatter_rhs(c->stream, (int64_t)c->tx.edge.size(), c->s_edge.p, c->s_col.p, c->s_val.p,
                     make_double2(0.0, -c->omega_mu0), ntx, c->b.p);
  if (pec_active(c)) launch_zero_rows(c->stream, (int64_t)c->pec_list.size(), c->pec_rows.p, ntx, c->b.p);
  MX_HIP_CHECK(hipGetLastError());
  int rc = fgmres(c, ntx, rtol, info);
  if (rc != MX_OK && rc != MX_ENOTCONV) return rc;
  const int nrx = rxs->n;
  CK(c->S.alloc((size_t)nrx * ntx));
  launch_receivers(c->stream, nrx, ntx, c->r_ptr.p, c->r_edge.p, c->r_val.p, c->x.p, c->S.p);
  MX_HIP_CHECK(hipGetLastError());
  if (S) CK(copy_out(c, S, c->S.p, (size_t)nrx * ntx * sizeof(double2)));
  if (E) CK(copy_out(c, E, c->x.p, blk * sizeof(double2)));
  CK(sync(c));
  c->have_forward = true;
  c->last_ntx = ntx;
  c->last_nrx = nrx;
  c->last_rtol = rtol;
  if (rc == MX_ENOTCONV) g_err = "FGMRES reached maxit";
  return rc;
}

int mx_set_krylov(mx_ctx* c, int32_t mode) {
  if (!c) return set_err(MX_EINVAL, "NULL context");
  if (mode != MX_KRYLOV_PSEUDO_BLOCK && mode != MX_KRYLOV_BLOCK && mode != MX_KRYLOV_BLOCK_CGS2)
    return set_err(MX_EINVAL, "unknown Krylov mode");
  c->krylov_mode = mode;
  return MX_OK;
}

int mx_set_ports(mx_ctx* c, int32_t nports, const mx_port* ports, int32_t pec) {
  if (!c || nports < 0 || (nports > 0 && !ports)) return set_err(MX_EINVAL, "bad arguments");
  if (nports > 256) return set_err(MX_EINVAL, "at most 256 ports");
  if (!c->have_mesh) return set_err(MX_ESTATE, "mx_assemble (with a mesh) must come first");
  for (int p = 0; p < nports; ++p) {
    const mx_port& q = ports[p];
    bool ok = q.a > 0 && q.b > 0 && std::isfinite(q.a) && std::isfinite(q.b) && std::isfinite(q.eps.re) &&
              std::isfinite(q.eps.im);
    double nn = 0, uu = 0, un = 0;
    for (int d = 0; d < 3; ++d) {
      ok = ok && std::isfinite(q.centre[d]) && std::isfinite(q.normal[d]) && std::isfinite(q.u[d]);
      nn += q.normal[d] * q.normal[d];
      uu += q.u[d] * q.u[d];
      un += q.u[d] * q.normal[d];
    }
    if (!ok || !(nn > 0) || !(uu - un * un / nn > 1e-12 * uu))
      return set_err(MX_EINVAL, "port " + std::to_string(p) + ": bad geometry or permittivity");
  }
  CK(use_device(c));
  const std::vector<mx_port> old_ports = c->ports;
  const bool old_pec = c->pec_walls;
  c->ports.assign(ports, ports + nports);
  c->pec_walls = nports > 0 && pec != 0;
  c->pec_list.clear();
  c->face_port.clear();
  if (nports > 0) {
    const int rc = build_ports(c);
    if (rc != MX_OK) {  // keep the previous configuration, which the operator still holds
      c->ports = old_ports;
      c->pec_walls = old_pec;
      c->pec_list.clear();
      c->face_port.clear();
      if (!c->ports.empty()) build_ports(c);
      return rc;
    }
  }
  c->local_ready = c->factored = false;
  c->have_forward = false;
  if (c->assembled) {
    CK(fill_pool(c));
    launch_gather_csr(c->stream, c->topo.nnz, c->cptr.p, c->csrc.p, c->pool.p, c->val.p);
    if (pec_active(c)) launch_pec_csr(c->stream, c->topo.ne, c->row_ptr.p, c->col.p, c->pec_flag.p, c->val.p);
    MX_HIP_CHECK(hipGetLastError());
  }
  return sync(c);
}

int mx_solve_ports(mx_ctx* c, double rtol, mx_c128* E, mx_c128* S, mx_solve_info* info) {
  if (!c) return set_err(MX_EINVAL, "NULL context");
  if (!(rtol > 0)) return set_err(MX_EINVAL, "rtol must be positive");
  if (c->ports.empty()) return set_err(MX_ESTATE, "no ports (mx_set_ports)");
  if (!c->factored) return set_err(MX_ESTATE, "mx_setup_schwarz (with factor=1) must come first");
  CK(use_device(c));
  const int np = (int)c->ports.size();
  // transmitters: b[e][p] = 2 j beta_p m_p[e]; receivers: m_p[e] / |e_p|^2
  std::vector<int32_t> col;
  std::vector<double2> bval, rval;
  for (int p = 0; p < np; ++p) {
    const double2 bt = port_beta(c->k0, c->ports[p]);
    const double2 g = make_double2(-2.0 * bt.y, 2.0 * bt.x);  // 2 j beta
    for (int64_t k = c->pm_ptr[p]; k < c->pm_ptr[p + 1]; ++k) {
      col.push_back(p);
      bval.push_back(make_double2(g.x * c->pm_val[k], g.y * c->pm_val[k]));
      rval.push_back(make_double2(c->pm_val[k] / c->pm_norm[p], 0.0));
    }
  }
  CK(c->pt_edge.upload(c->pm_edge, c->stream));
  CK(c->pt_col.upload(col, c->stream));
  CK(c->pt_val.upload(bval, c->stream));
  CK(c->pr_ptr.upload(c->pm_ptr, c->stream));
  CK(c->pr_edge.upload(c->pm_edge, c->stream));
  CK(c->pr_val.upload(rval, c->stream));
  CK(ensure_workspace(c, np, c->restart));
  const int64_t blk = c->topo.ne * (int64_t)np;
  launch_fill_zero<double2>(c->stream, blk, c->b.p);
  launch_scatter_rhs(c->stream, (int64_t)c->pm_edge.size(), c->pt_edge.p, c->pt_col.p, c->pt_val.p,
                     make_double2(1.0, 0.0), np, c->b.p);
  MX_HIP_CHECK(hipGetLastError());
  int rc = fgmres(c, np, rtol, info);
  if (rc != MX_OK && rc != MX_ENOTCONV) return rc;
  CK(c->S.alloc((size_t)np * np));
  launch_receivers(c->stream, np, np, c->pr_ptr.p, c->pr_edge.p, c->pr_val.p, c->x.p, c->S.p);
  MX_HIP_CHECK(hipGetLastError());
  std::vector<double2> hS((size_t)np * np);
  MX_HIP_CHECK(hipMemcpyAsync(hS.data(), c->S.p, hS.size() * sizeof(double2), hipMemcpyDeviceToHost, c->stream));
  CK(sync(c));
  for (int p = 0; p < np; ++p) hS[(size_t)p * np + p].x -= 1.0;
  if (S && is_device_ptr(S))
    MX_HIP_CHECK(hipMemcpyAsync(S, hS.data(), hS.size() * sizeof(double2), hipMemcpyHostToDevice, c->stream));
  else if (S)
    std::memcpy(S, hS.data(), hS.size() * sizeof(double2));
  if (E) CK(copy_out(c, E, c->x.p, blk * sizeof(double2)));
  CK(sync(c));
  c->have_forward = false;  // the adjoint gradient is defined for point sources
  c->tx = SourceSet();
  return rc;
}

int mx_gradient(mx_ctx* c, const mx_c128* S_meas, const double* w, double alpha, mx_c128* grad, double* J,
                mx_solve_info* info) {
  if (!c || !S_meas || !w || !grad || !J) return set_err(MX_EINVAL, "NULL argument");
  if (!c->have_forward || !c->factored) return set_err(MX_ESTATE, "mx_gradient needs a preceding mx_solve");
  if (c->eps_kind != MX_EPS_P1) return set_err(MX_EINVAL, "the gradient is defined for per-vertex permittivity");
  if (!(alpha >= 0) || !std::isfinite(alpha)) return set_err(MX_EINVAL, "alpha must be finite and >= 0");
  CK(use_device(c));
  const Topology& T = c->topo;
  const int ntx = c->last_ntx, nrx = c->last_nrx;
  const int64_t blk = T.ne * (int64_t)ntx;
  // misfit d = S - S_meas and its cost (host, nrx x ntx)
  std::vector<double2> Sh((size_t)nrx * ntx);
  MX_HIP_CHECK(hipMemcpyAsync(Sh.data(), c->S.p, Sh.size() * sizeof(double2), hipMemcpyDeviceToHost, c->stream));
  CK(sync(c));
  double Jm = 0;
  std::vector<std::pair<int64_t, double2>> acc;
  for (int i = 0; i < nrx; ++i)
    for (int j = 0; j < ntx; ++j) {
      const size_t o = (size_t)i * ntx + j;
      const double dr = Sh[o].x - S_meas[o].re, di = Sh[o].y - S_meas[o].im;
      Jm += 0.5 * w[o] * (dr * dr + di * di);
      // adjoint source of transmitter j: w_ij conj(d_ij) r_i
      const double cr = w[o] * dr, ci = -w[o] * di;
      for (int64_t k = c->rx.ptr[i]; k < c->rx.ptr[i + 1]; ++k) {
        const double2 v = c->rx.val[k];
        acc.push_back({(int64_t)c->rx.edge[k] * ntx + j, make_double2(cr * v.x - ci * v.y, cr * v.y + ci * v.x)});
      }
    }
  std::stable_sort(acc.begin(), acc.end(), [](const auto& a, const auto& b) { return a.first < b.first; });
  std::vector<int32_t> ae, ac;
  std::vector<double2> av;
  for (size_t a = 0; a < acc.size();) {
    size_t b = a;
    double2 v = make_double2(0, 0);
    while (b < acc.size() && acc[b].first == acc[a].first) {
      v.x += acc[b].second.x;
      v.y += acc[b].second.y;
      ++b;
    }
    ae.push_back((int32_t)(acc[a].first / ntx));
    ac.push_back((int32_t)(acc[a].first % ntx));
    av.push_back(v);
    a = b;
  }
  CK(c->a_edge.upload(ae, c->stream));
  CK(c->a_col.upload(ac, c->stream));
  CK(c->a_val.upload(av, c->stream));
  // keep the forward fields, solve the adjoint problems with the same factors
  CK(c->U_fwd.alloc(blk));
  MX_HIP_CHECK(hipMemcpyAsync(c->U_fwd.p, c->x.p, blk * sizeof(double2), hipMemcpyDeviceToDevice, c->stream));
  launch_fill_zero<double2>(c->stream, blk, c->b.p);
  launch_scatter_rhs(c->stream, (int64_t)ae.size(), c->a_edge.p, c->a_col.p, c->a_val.p, make_double2(1.0, 0.0),
                     ntx, c->b.p);
  MX_HIP_CHECK(hipGetLastError());
  int rc = fgmres(c, ntx, c->last_rtol, info);
  if (rc != MX_OK && rc != MX_ENOTCONV) return rc;
  // gradient: per-tetrahedron contraction, then a per-vertex gather
  if (!c->t2e.p) CK(c->t2e.upload(T.t2e, c->stream));
  if (!c->v2t.p) {
    CK(c->v2t.upload(T.v2t, c->stream));
    CK(c->v2t_ptr.upload(T.v2t_ptr, c->stream));
  }
  CK(c->gt.alloc(4 * (size_t)T.nt));
  CK(c->rt.alloc(4 * (size_t)T.nt));
  CK(c->gradv.alloc((size_t)T.nv));
  CK(c->keps.alloc((size_t)T.nv));
  const double k0sq = c->k0 * c->k0;
  launch_grad_tet(c->stream, T.nt, c->ts.p, c->xyz.p, c->t2e.p, c->x.p, c->U_fwd.p, ntx, c->eps.p, k0sq, c->gt.p,
                  c->rt.p);
  launch_grad_vertex(c->stream, T.nv, c->v2t_ptr.p, c->v2t.p, c->ts.p, c->gt.p, c->rt.p, alpha * k0sq * k0sq,
                     c->gradv.p, c->keps.p);
  MX_HIP_CHECK(hipGetLastError());
  CK(copy_out(c, grad, c->gradv.p, (size_t)T.nv * sizeof(double2)));
  std::vector<double2> ke(T.nv), ep(T.nv);
  MX_HIP_CHECK(hipMemcpyAsync(ke.data(), c->keps.p, T.nv * sizeof(double2), hipMemcpyDeviceToHost, c->stream));
  MX_HIP_CHECK(hipMemcpyAsync(ep.data(), c->eps.p, T.nv * sizeof(double2), hipMemcpyDeviceToHost, c->stream));
  // restore the forward fields as the current solution
  MX_HIP_CHECK(hipMemcpyAsync(c->x.p, c->U_fwd.p, blk * sizeof(double2), hipMemcpyDeviceToDevice, c->stream));
  CK(sync(c));
  double R = 0;
  for (int64_t n = 0; n < T.nv; ++n) R += ep[n].x * ke[n].x + ep[n].y * ke[n].y;
  *J = Jm + alpha * 0.5 * k0sq * k0sq * R;
  if (rc == MX_ENOTCONV) g_err = "adjoint FGMRES reached maxit";
  return rc;
}

int mx_apply_operator(mx_ctx* c, const mx_c128* X, mx_c128* Y, int32_t nrhs) {
  if (!c || !X || !Y || nrhs <= 0) return set_err(MX_EINVAL, "bad arguments");
  if (!c->assembled) return set_err(MX_ESTATE, "mx_assemble must come first");
  CK(use_device(c));
  const size_t bytes = (size_t)c->topo.ne * nrhs * sizeof(double2);
  DBuf<double2> xin, yout;
  CK(xin.alloc((size_t)c->topo.ne * nrhs));
  CK(yout.alloc((size_t)c->topo.ne * nrhs));
  CK(copy_in(c, xin.p, X, bytes));
  CK(spmm(c, xin.p, yout.p, nrhs));
  CK(copy_out(c, Y, yout.p, bytes));
  CK(sync(c));
  return MX_OK;
}

int mx_apply_preconditioner(mx_ctx* c, const mx_c128* X, mx_c128* Zo, int32_t nrhs) {
  if (!c || !X || !Zo || nrhs <= 0) return set_err(MX_EINVAL, "bad arguments");
  if (!c->factored) return set_err(MX_ESTATE, "mx_setup_schwarz (with factor=1) must come first");
  if (nrhs > 256) return set_err(MX_EINVAL, "at most 256 right-hand sides");
  CK(use_device(c));
  const size_t bytes = (size_t)c->topo.ne * nrhs * sizeof(double2);
  DBuf<double2> xin, zout;
  CK(xin.alloc((size_t)c->topo.ne * nrhs));
  CK(zout.alloc((size_t)c->topo.ne * nrhs));
  CK(c->xloc.alloc((size_t)c->dec.vec_off[c->dec.nsub] * nrhs * elem_bytes(c->precision)));
  CK(copy_in(c, xin.p, X, bytes));
  if (learned_ready(c)) {
    DBuf<double2> w;
    CK(w.alloc((size_t)c->topo.ne * nrhs));
    CK(ensure_learned_ws(c, nrhs));
    c->coarse_off_now = false;
    CK(precond_learned(c, xin.p, zout.p, w.p, nrhs));
  } else {
    CK(apply_precond(c, xin.p, zout.p, nrhs));
  }
  CK(copy_out(c, Zo, zout.p, bytes));
  CK(sync(c));
  return MX_OK;
}

int mx_apply_preconditioner_noalloc(mx_ctx* c, const mx_c128* X, mx_c128* Zo, int32_t nrhs) {
  if (!c || !X || !Zo || nrhs <= 0) return set_err(MX_EINVAL, "bad arguments");
  if (nrhs > 256) return set_err(MX_EINVAL, "at most 256 right-hand sides");
  if (!c->factored) return set_err(MX_ESTATE, "mx_setup_schwarz (with factor=1) must come first");
  if (learned_ready(c))
    return set_err(MX_ESTATE, "the learned term needs allocated buffers: use mx_apply_preconditioner");
  if (!c->scratch_dev) return set_err(MX_ESTATE, "no scratch address for this device");
  const size_t need = (size_t)c->dec.vec_off[c->dec.nsub] * nrhs * elem_bytes(c->precision);
  if (need > kScratchBytes)
    return set_err(MX_EINVAL, "needs " + std::to_string(need) + " bytes of scratch, the fixed buffer holds " +
                                  std::to_string(kScratchBytes) + ": use fewer right-hand sides per call");
  CK(use_device(c));
  if (!is_device_ptr(X) || !is_device_ptr(Zo)) return set_err(MX_EINVAL, "X and Z must be device pointers");
  CK(apply_precond(c, (const double2*)X, (double2*)Zo, nrhs, nullptr, c->scratch_dev));
  return MX_OK;
}

int mx_get_sizes(mx_ctx* c, mx_sizes* o) {
  if (!c || !o) return set_err(MX_EINVAL, "NULL argument");
  std::memset(o, 0, sizeof(*o));
  if (c->have_mesh) {
    o->nv = c->topo.nv;
    o->nt = c->topo.nt;
    o->ne = c->topo.ne;
    o->nnz = c->topo.nnz;
    o->nbface = c->topo.nbf;
  }
  if (c->have_dec) {
    o->nsub = c->dec.nsub;
    o->overlap = c->dec.overlap;
    o->ncolour = c->dec.ncolour;
    o->sum_ni = c->dec.dof_ptr[c->dec.nsub];
    o->sum_Ni2 = c->dec.mat_off[c->dec.nsub];
    o->nb = c->dec.nb;
  }
  if (c->factored) {
    o->lu_tiles = c->lu_tiles;
    o->trsm_tiles_lower = c->trsm_tiles_l;
    o->trsm_tiles_upper = c->trsm_tiles_u;
  }
  return MX_OK;
}

int mx_get_topology(mx_ctx* c, int32_t* edges, int32_t* t2e, int64_t* row_ptr, int32_t* col) {
  if (!c) return set_err(MX_EINVAL, "NULL context");
  if (!c->have_mesh) return set_err(MX_ESTATE, "no mesh");
  const Topology& T = c->topo;
  if (edges) std::memcpy(edges, T.edges.data(), T.edges.size() * sizeof(int32_t));
  if (t2e) std::memcpy(t2e, T.t2e.data(), T.t2e.size() * sizeof(int32_t));
  if (row_ptr) std::memcpy(row_ptr, T.row_ptr.data(), T.row_ptr.size() * sizeof(int64_t));
  if (col) std::memcpy(col, T.col.data(), T.col.size() * sizeof(int32_t));
  return MX_OK;
}

int mx_get_matrix_values(mx_ctx* c, mx_c128* v) {
  if (!c || !v) return set_err(MX_EINVAL, "NULL argument");
  if (!c->assembled) return set_err(MX_ESTATE, "not assembled");
  CK(use_device(c));
  MX_HIP_CHECK(hipMemcpyAsync(v, c->val.p, c->topo.nnz * sizeof(double2), hipMemcpyDeviceToHost, c->stream));
  return sync(c);
}

int mx_get_partition(mx_ctx* c, int32_t* part, int64_t* dof_ptr, int32_t* dofs, int32_t* pu_w, int32_t* colour) {
  if (!c) return set_err(MX_EINVAL, "NULL context");
  if (!c->have_dec) return set_err(MX_ESTATE, "no decomposition");
  const Decomposition& D = c->dec;
  if (part) std::memcpy(part, D.part.data(), D.part.size() * sizeof(int32_t));
  if (dof_ptr) std::memcpy(dof_ptr, D.dof_ptr.data(), D.dof_ptr.size() * sizeof(int64_t));
  if (dofs) std::memcpy(dofs, D.dofs.data(), D.dofs.size() * sizeof(int32_t));
  if (pu_w) std::memcpy(pu_w, D.w.data(), D.w.size() * sizeof(int32_t));
  if (colour) std::memcpy(colour, D.colour.data(), D.colour.size() * sizeof(int32_t));
  return MX_OK;
}

int mx_get_local_matrix(mx_ctx* c, int32_t i, mx_c128* B) {
  if (!c || !B) return set_err(MX_EINVAL, "NULL argument");
  if (!c->have_dec || !c->local_ready || c->factored)
    return set_err(MX_ESTATE, "needs mx_setup_schwarz with factor = 0");
  if (i < 0 || i >= c->dec.nsub) return set_err(MX_EINVAL, "subdomain index out of range");
  CK(use_device(c));
  const Decomposition& D = c->dec;
  const int n = (int)(D.dof_ptr[i + 1] - D.dof_ptr[i]);
  const int N = D.Npad[i];
  DBuf<double2> tmp;
  CK(tmp.alloc((size_t)n * n));
  const unsigned g = (unsigned)(((int64_t)n * n + 255) / 256);
  if (c->precision == MX_PREC_C64)
    hipLaunchKernelGGL(k_extract_local<float2>, dim3(g), dim3(256), 0, c->stream, n, N,
                       (const float2*)c->factors.p + D.mat_off[i], tmp.p);
  else
    hipLaunchKernelGGL(k_extract_local<double2>, dim3(g), dim3(256), 0, c->stream, n, N,
                       (const double2*)c->factors.p + D.mat_off[i], tmp.p);
  MX_HIP_CHECK(hipGetLastError());
  std::vector<double2> h((size_t)n * n);
  MX_HIP_CHECK(hipMemcpyAsync(h.data(), tmp.p, h.size() * sizeof(double2), hipMemcpyDeviceToHost, c->stream));
  CK(sync(c));
  // dense rows are in the subdomain's reverse Cuthill-McKee order: back to
  // the sorted DOF order of the interface
  const int32_t* lp = D.lpos.data() + D.dof_ptr[i];
  for (int a = 0; a < n; ++a)
    for (int b = 0; b < n; ++b) {
      const double2 v = h[(size_t)lp[a] * n + lp[b]];
      B[(size_t)a * n + b].re = v.x;
      B[(size_t)a * n + b].im = v.y;
    }
  return MX_OK;
}


int mx_coarse_init(mx_ctx* c, uint64_t seed) {
  if (!c) return set_err(MX_EINVAL, "NULL context");
  CK(use_device(c));
  std::vector<float> th(NL.total, 0.f);
  std::mt19937_64 rng(seed);
  std::normal_distribution<double> nd(0.0, 1.0);
  auto fill = [&](int64_t off, int rows, int cols, double scale) {
    for (int64_t k = 0; k < (int64_t)rows * cols; ++k) th[off + k] = (float)(scale * nd(rng) / std::sqrt((double)cols));
  };
  for (int l = 0; l < 4; ++l) fill(NL.W[l], NW, l == 0 ? NIN : NW, 1.0);
  fill(NL.Ws1, NW, NW, 1.0);
  fill(NL.Wn1, NW, NW, 1.0);
  fill(NL.Ws2, NIN, NW, 0.1);
  fill(NL.Wn2, NIN, NW, 0.1);
  CK(c->theta.upload(th, c->stream));
  CK(c->gtheta.alloc(NL.total));
  CK(c->adam_m.alloc(NL.total));
  CK(c->adam_v.alloc(NL.total));
  std::vector<float> z(NL.total, 0.f);
  MX_HIP_CHECK(hipMemcpyAsync(c->adam_m.p, z.data(), z.size() * 4, hipMemcpyHostToDevice, c->stream));
  MX_HIP_CHECK(hipMemcpyAsync(c->adam_v.p, z.data(), z.size() * 4, hipMemcpyHostToDevice, c->stream));
  c->adam_t = 0;
  c->sx = c->sy = 1.0;
  c->coarse_weights = true;
  return sync(c);
}

int64_t mx_coarse_num_params(void) { return NL.total; }

int mx_coarse_set_weights(mx_ctx* c, const float* theta, int64_t n, double in_scale, double out_scale) {
  if (!c || !theta) return set_err(MX_EINVAL, "NULL argument");
  if (n != NL.total) return set_err(MX_EINVAL, "expected " + std::to_string(NL.total) + " parameters");
  if (!(in_scale > 0) || !(out_scale > 0)) return set_err(MX_EINVAL, "scales must be positive");
  CK(use_device(c));
  if (!c->coarse_weights) CK(mx_coarse_init(c, 0));
  MX_HIP_CHECK(hipMemcpyAsync(c->theta.p, theta, n * sizeof(float), hipMemcpyHostToDevice, c->stream));
  launch_fill_zero<float>(c->stream, NL.total, c->adam_m.p);
  launch_fill_zero<float>(c->stream, NL.total, c->adam_v.p);
  c->adam_t = 0;
  c->sx = in_scale;
  c->sy = out_scale;
  MX_HIP_CHECK(hipGetLastError());
  return sync(c);
}
int mx_coarse_adam_step(mx_ctx* c, const float* grad, int64_t n, double lr) {
  if (!c || !grad) return set_err(MX_EINVAL, "NULL argument");
  if (n != NL.total) return set_err(MX_EINVAL, "expected " + std::to_string(NL.total) + " gradient values");
  if (!(lr > 0) || !std::isfinite(lr)) return set_err(MX_EINVAL, "lr must be positive");
  if (!c->coarse_weights) return set_err(MX_ESTATE, "call mx_coarse_init or mx_coarse_set_weights first");
  CK(use_device(c));
  CK(copy_in(c, c->gtheta.p, grad, n * sizeof(float)));
  launch_adam(c->stream, NL.total, c->theta.p, c->gtheta.p, c->adam_m.p, c->adam_v.p, (float)lr, 0.9f, 0.999f, 1e-8f,
              ++c->adam_t);
  MX_HIP_CHECK(hipGetLastError());
  return sync(c);
}

int mx_coarse_get_weights(mx_ctx* c, float* theta, int64_t n, double* in_scale, double* out_scale) {
  if (!c || !theta) return set_err(MX_EINVAL, "NULL argument");
  if (!c->coarse_weights) return set_err(MX_ESTATE, "no network weights");
  if (n != NL.total) return set_err(MX_EINVAL, "expected " + std::to_string(NL.total) + " parameters");
  CK(use_device(c));
  MX_HIP_CHECK(hipMemcpyAsync(theta, c->theta.p, n * sizeof(float), hipMemcpyDeviceToHost, c->stream));
  if (in_scale) *in_scale = c->sx;
  if (out_scale) *out_scale = c->sy;
  return sync(c);
}

int mx_coarse_features(mx_ctx* c, const mx_c128* v, int32_t nrhs, float* X) {
  if (!c || !v || !X || nrhs <= 0 || nrhs > 256) return set_err(MX_EINVAL, "bad arguments");
  if (!c->coarse_geom) return set_err(MX_ESTATE, "needs mx_setup_schwarz with opts.coarse = 1");
  CK(use_device(c));
  const Decomposition& D = c->dec;
  DBuf<double2> vin;
  DBuf<float> Xd;
  CK(vin.alloc((size_t)c->topo.ne * nrhs));
  CK(Xd.alloc((size_t)nrhs * D.nsub * NIN));
  CK(copy_in(c, vin.p, v, (size_t)c->topo.ne * nrhs * sizeof(double2)));
  CK(c->normpart.alloc((size_t)dot_blocks(c->topo.ne) * nrhs));
  launch_norm(c->stream, c->topo.ne, nrhs, vin.p, c->normpart.p, c->cscale.p);
  launch_scale_rhs_norm(c, nrhs);
  launch_pool(c->stream, D.nsub, c->dof_ptr.p, c->dofs.p, c->cP.p, nullptr, vin.p, nrhs, c->cscale.p, Xd.p, c->cpart.p);
  MX_HIP_CHECK(hipGetLastError());
  MX_HIP_CHECK(hipMemcpyAsync(X, Xd.p, (size_t)nrhs * D.nsub * NIN * 4, hipMemcpyDeviceToHost, c->stream));
  return sync(c);
}

int mx_coarse_hidden(mx_ctx* c, const float* X, int32_t ngraph, float* H, float* out) {
  if (!c || !X || !H || !out || ngraph <= 0) return set_err(MX_EINVAL, "bad arguments");
  if (!c->have_dec || !c->coarse_geom || !c->coarse_weights) return set_err(MX_ESTATE, "needs coarse set-up and weights");
  CK(use_device(c));
  const int64_t rows = (int64_t)ngraph * c->dec.nsub;
  NetBufs B;
  CK(net_bufs(c, rows, B));
  MX_HIP_CHECK(hipMemcpyAsync(B.X, X, rows * NIN * 4, hipMemcpyHostToDevice, c->stream));
  net_forward(c, ngraph, B);
  MX_HIP_CHECK(hipGetLastError());
  const float* hs[5] = {B.H[0], B.H[1], B.H[2], B.H[3], B.H5};
  for (int l = 0; l < 5; ++l)
    MX_HIP_CHECK(hipMemcpyAsync(H + (size_t)l * rows * NW, hs[l], rows * NW * 4, hipMemcpyDeviceToHost, c->stream));
  MX_HIP_CHECK(hipMemcpyAsync(out, B.OUT, rows * NIN * 4, hipMemcpyDeviceToHost, c->stream));
  return sync(c);
}
int mx_coarse_forward(mx_ctx* c, const float* X, int32_t ngraph, float* out) {
  if (!c || !X || !out || ngraph <= 0) return set_err(MX_EINVAL, "bad arguments");
  if (!c->have_dec || !c->coarse_geom || !c->coarse_weights) return set_err(MX_ESTATE, "needs coarse set-up and weights");
  CK(use_device(c));
  const int64_t rows = (int64_t)ngraph * c->dec.nsub;
  NetBufs B;
  CK(net_bufs(c, rows, B));
  MX_HIP_CHECK(hipMemcpyAsync(B.X, X, rows * NIN * 4, hipMemcpyHostToDevice, c->stream));
  net_forward(c, ngraph, B);
  MX_HIP_CHECK(hipGetLastError());
  MX_HIP_CHECK(hipMemcpyAsync(out, B.OUT, rows * NIN * 4, hipMemcpyDeviceToHost, c->stream));
  return sync(c);
}

double mse_loss(mx_ctx* c, int64_t n, NetBufs& B, const float* Ydev) {
  (void)c->msepart.alloc(mse_blocks());
  launch_mse(c->stream, n, B.OUT, Ydev, B.dOUT, c->msepart.p);
  std::vector<double> part(mse_blocks());
  (void)hipMemcpyAsync(part.data(), c->msepart.p, part.size() * sizeof(double), hipMemcpyDeviceToHost, c->stream);
  (void)hipStreamSynchronize(c->stream);
  double sum = 0;
  for (double v : part) sum += v;
  return sum / (double)n;
}

int mx_coarse_loss_grad(mx_ctx* c, const float* X, const float* Y, int32_t ngraph, double* loss, float* grad) {
  if (!c || !X || !Y || !loss || !grad || ngraph <= 0) return set_err(MX_EINVAL, "bad arguments");
  if (!c->have_dec || !c->coarse_geom || !c->coarse_weights) return set_err(MX_ESTATE, "needs coarse set-up and weights");
  CK(use_device(c));
  const int64_t rows = (int64_t)ngraph * c->dec.nsub;
  NetBufs B;
  CK(net_bufs(c, rows, B));
  MX_HIP_CHECK(hipMemcpyAsync(B.X, X, rows * NIN * 4, hipMemcpyHostToDevice, c->stream));
  MX_HIP_CHECK(hipMemcpyAsync(B.dOUT, Y, rows * NIN * 4, hipMemcpyHostToDevice, c->stream));
  net_forward(c, ngraph, B);
  *loss = mse_loss(c, rows * NIN, B, B.dOUT);
  net_backward(c, ngraph, B);
  MX_HIP_CHECK(hipGetLastError());
  MX_HIP_CHECK(hipMemcpyAsync(grad, c->gtheta.p, NL.total * 4, hipMemcpyDeviceToHost, c->stream));
  return sync(c);
}

int mx_coarse_clear(mx_ctx* c) {
  if (!c) return set_err(MX_EINVAL, "NULL context");
  c->ds_graphs = 0;
  return MX_OK;
}

int mx_coarse_collect(mx_ctx* c, const mx_sources* tx, int32_t snap_every, int32_t max_snapshots, double rtol_exact,
                      int32_t* nsnap) {
  if (!c || !tx || snap_every < 1 || max_snapshots < 1 || !(rtol_exact > 0)) return set_err(MX_EINVAL, "bad arguments");
  if (!c->factored) return set_err(MX_ESTATE, "mx_setup_schwarz (with factor=1) must come first");
  CK(use_device(c));
  if (!c->coarse_geom) CK(coarse_prepare(c));
  const Decomposition& D = c->dec;
  const int ntx = tx->n;
  if (ntx > 256) return set_err(MX_EINVAL, "at most 256 transmitters");
  CK(build_sources(c, tx, c->tx));
  {
    std::vector<int32_t> colv(c->tx.edge.size());
    for (int j = 0; j < ntx; ++j)
      for (int64_t k = c->tx.ptr[j]; k < c->tx.ptr[j + 1]; ++k) colv[k] = j;
    CK(c->s_edge.upload(c->tx.edge, c->stream));
    CK(c->s_col.upload(colv, c->stream));
    CK(c->s_val.upload(c->tx.val, c->stream));
  }
  const bool use_save = c->coarse_use;
  c->coarse_use = false;
  CK(ensure_workspace(c, ntx, c->restart));
  const int64_t blk = c->topo.ne * (int64_t)ntx;
  launch_fill_zero<double2>(c->stream, blk, c->b.p);
  launch_scatter_rhs(c->stream, (int64_t)c->tx.edge.size(), c->s_edge.p, c->s_col.p, c->s_val.p,
                     make_double2(0.0, -c->omega_mu0), ntx, c->b.p);
  int rc = fgmres(c, ntx, rtol_exact, nullptr);
  if (rc != MX_OK) { c->coarse_use = use_save; return rc; }
  DBuf<double2> xs;
  CK(xs.alloc(blk));
  MX_HIP_CHECK(hipMemcpyAsync(xs.p, c->x.p, blk * sizeof(double2), hipMemcpyDeviceToDevice, c->stream));
  // grow the data set
  const int64_t per_graph = (int64_t)D.nsub * NIN;
  const int64_t need = c->ds_graphs + (int64_t)max_snapshots * ntx;
  if (need > c->ds_cap) {
    DBuf<float> nx, ny;
    CK(nx.alloc((size_t)need * per_graph));
    CK(ny.alloc((size_t)need * per_graph));
    if (c->ds_graphs) {
      MX_HIP_CHECK(hipMemcpyAsync(nx.p, c->dsX.p, c->ds_graphs * per_graph * 4, hipMemcpyDeviceToDevice, c->stream));
      MX_HIP_CHECK(hipMemcpyAsync(ny.p, c->dsY.p, c->ds_graphs * per_graph * 4, hipMemcpyDeviceToDevice, c->stream));
    }
    CK(sync(c));
    std::swap(c->dsX.p, nx.p); std::swap(c->dsX.n, nx.n);
    std::swap(c->dsY.p, ny.p); std::swap(c->dsY.n, ny.n);
    c->ds_cap = need;
  }
  NetBufs B;
  CK(net_bufs(c, (int64_t)ntx * D.nsub, B));
  CK(ensure_workspace(c, ntx, snap_every));
  DBuf<double> Dw;
  CK(Dw.upload(D.D, c->stream));
  int count = 0;
  std::function<int()> cb = [&]() -> int {
    if (count >= max_snapshots) return MX_OK;
    hipStream_t s = c->stream;
    float* Xo = c->dsX.p + c->ds_graphs * per_graph;
    float* Yo = c->dsY.p + c->ds_graphs * per_graph;
    launch_norm(s, c->topo.ne, ntx, c->r.p, c->normpart.p, c->cscale.p);
    launch_scale_rhs_norm(c, ntx);
    launch_pool(s, D.nsub, c->dof_ptr.p, c->dofs.p, c->cP.p, nullptr, c->r.p, ntx, c->cscale.p, Xo, c->cpart.p);
    double2* mr = c->Z.p;
    double2* t = c->V.p + blk;
    CK(apply_precond(c, c->r.p, mr, ntx));
    hipLaunchKernelGGL(k_axpy_err, dim3((unsigned)((blk + 255) / 256)), dim3(256), 0, s, blk, xs.p, c->x.p, mr, t);
    launch_pool(s, D.nsub, c->dof_ptr.p, c->dofs.p, c->cP.p, Dw.p, t, ntx, c->cscale.p, B.X, c->cpart.p);
    launch_gapply(s, D.nsub, ntx, c->cG.p, B.X, Yo);
    MX_HIP_CHECK(hipGetLastError());
    c->ds_graphs += ntx;
    ++count;
    return MX_OK;
  };
  rc = fgmres(c, ntx, rtol_exact, nullptr, &cb);
  c->coarse_use = use_save;
  CK(ensure_workspace(c, ntx, c->restart));
  if (nsnap) *nsnap = count;
  CK(sync(c));
  return rc == MX_ENOTCONV ? MX_OK : rc;
}

int mx_coarse_train(mx_ctx* c, int32_t epochs, int32_t batch_graphs, double lr, uint64_t seed, double* loss_hist) {
  if (!c || epochs < 1 || batch_graphs < 1 || !(lr > 0)) return set_err(MX_EINVAL, "bad arguments");
  if (!c->coarse_weights) return set_err(MX_ESTATE, "call mx_coarse_init first");
  if (c->ds_graphs < 1) return set_err(MX_ESTATE, "no training data (mx_coarse_collect)");
  CK(use_device(c));
  const Decomposition& D = c->dec;
  const int64_t per_graph = (int64_t)D.nsub * NIN;
  // input / output scales from (up to) the first 64 graphs
  {
    const int64_t ng = std::min<int64_t>(64, c->ds_graphs);
    std::vector<float> hx(ng * per_graph), hy(ng * per_graph);
    MX_HIP_CHECK(hipMemcpyAsync(hx.data(), c->dsX.p, hx.size() * 4, hipMemcpyDeviceToHost, c->stream));
    MX_HIP_CHECK(hipMemcpyAsync(hy.data(), c->dsY.p, hy.size() * 4, hipMemcpyDeviceToHost, c->stream));
    CK(sync(c));
    double a = 0, b = 0;
    for (size_t k = 0; k < hx.size(); ++k) { a += (double)hx[k] * hx[k]; b += (double)hy[k] * hy[k]; }
    c->sx = std::sqrt(a / hx.size());
    c->sy = std::sqrt(b / hy.size());
    if (!(c->sx > 0)) c->sx = 1;
    if (!(c->sy > 0)) c->sy = 1;
  }
  const int bg = (int)std::min<int64_t>(batch_graphs, c->ds_graphs);
  NetBufs B;
  CK(net_bufs(c, (int64_t)bg * D.nsub, B));
  CK(c->bgraph.alloc(bg));
  std::mt19937_64 rng(seed);
  std::vector<int32_t> perm(c->ds_graphs);
  for (int64_t g = 0; g < c->ds_graphs; ++g) perm[g] = (int32_t)g;
  for (int ep = 0; ep < epochs; ++ep) {
    std::shuffle(perm.begin(), perm.end(), rng);
    double lsum = 0;
    int nb = 0;
    for (int64_t b0 = 0; b0 + bg <= c->ds_graphs; b0 += bg) {
      MX_HIP_CHECK(hipMemcpyAsync(c->bgraph.p, perm.data() + b0, bg * 4, hipMemcpyHostToDevice, c->stream));
      const int rows = bg * D.nsub;
      launch_gather_rows(c->stream, rows, NIN, c->bgraph.p, D.nsub, c->dsX.p, B.X);
      launch_gather_rows(c->stream, rows, NIN, c->bgraph.p, D.nsub, c->dsY.p, B.dOUT);
      launch_scale_f(c->stream, (int64_t)rows * NIN, B.X, (float)(1.0 / c->sx));
      launch_scale_f(c->stream, (int64_t)rows * NIN, B.dOUT, (float)(1.0 / c->sy));
      net_forward(c, bg, B);
      lsum += mse_loss(c, (int64_t)rows * NIN, B, B.dOUT);
      net_backward(c, bg, B);
      launch_adam(c->stream, NL.total, c->theta.p, c->gtheta.p, c->adam_m.p, c->adam_v.p, (float)lr, 0.9f, 0.999f,
                  1e-8f, ++c->adam_t);
      MX_HIP_CHECK(hipGetLastError());
      ++nb;
    }
    if (loss_hist) loss_hist[ep] = nb ? lsum / nb : 0.0;
  }
  return sync(c);
}

int mx_point_functionals(mx_ctx* c, const mx_sources* pts, mx_c128* R) {
  if (!c || !pts || !R) return set_err(MX_EINVAL, "NULL argument");
  if (!c->have_mesh) return set_err(MX_ESTATE, "no mesh");
  SourceSet s;
  CK(build_sources(c, pts, s));
  const int n = pts->n;
  std::memset(R, 0, (size_t)c->topo.ne * n * sizeof(mx_c128));
  for (int j = 0; j < n; ++j)
    for (int64_t k = s.ptr[j]; k < s.ptr[j + 1]; ++k) {
      R[(size_t)s.edge[k] * n + j].re = s.val[k].x;
      R[(size_t)s.edge[k] * n + j].im = s.val[k].y;
    }
  return MX_OK;
}

}  // extern "C"
