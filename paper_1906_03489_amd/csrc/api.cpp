// C ABI of the library: argument validation, handle management and dispatch.
// Every entry point validates before touching the device and converts every
// failure into an nk_status with a thread-local message.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <map>
#include <mutex>
#include <numeric>
#include <sstream>
#include <string>
#include <thread>
#include <tuple>
#include <vector>

#include "nk_internal.h"
#include "system.h"
#include "tiles.h"

namespace nk {

static thread_local std::string g_err;

void set_error(const std::string& msg) { g_err = msg; }

nk_status fail(nk_status st, const std::string& msg) {
  g_err = msg;
  return st;
}

nk_status hip_fail(hipError_t e, const char* what) {
  std::string m = std::string(what) + ": " + hipGetErrorString(e);
  g_err = m;
  return e == hipErrorOutOfMemory ? NK_ENOMEM : NK_EHIP;
}

bool op_supported(int dim, int P, int Q) {
  return (dim == 2 || dim == 3) && P >= kMinP && P <= kMaxP && Q == P + 2;
}

hipError_t launch_op3(nk_dtype t, const OpArgs& a) {
  if (a.nelem == 0) return hipSuccess;
  switch (a.P) {
    case 1: case 2: case 3: case 4: return launch_op3_set0(t, a);
    case 5: return launch_op3_set1(t, a);
    case 6: return launch_op3_set2(t, a);
    case 7: return launch_op3_set3(t, a);
    case 8: return launch_op3_set4(t, a);
    case 9: return launch_op3_set5(t, a);
    case 10: return launch_op3_set6(t, a);
  }
  return hipErrorInvalidValue;
}

static int vector_tile_count(int op, int dim, int P);

static hipError_t launch_op(int dim, nk_dtype t, const OpArgs& a) {
  if (a.nelem == 0) return hipSuccess;
  if ((a.op == OP_HELM || a.op == OP_HELM_ASM) && mfma_supported(dim, a.P) &&
      a.tile == vector_tile_count(OP_HELM, dim, a.P))
    return launch_helm_mfma(t, a);
  return dim == 3 ? launch_op3(t, a) : launch_op2(t, a);
}

// ------------------------------------------------------------- tile choice
static std::atomic<int> g_tile[OP_COUNT][2][kMaxP + 1][2];
// set once a caller chose the Helmholtz tile explicitly (or NK_TILE is set):
// systems then use that choice instead of timing their own operator
static std::atomic<bool> g_tile_forced[2][kMaxP + 1][2];

// vector-ALU tile candidates (elements per block)
static int vector_tile_count(int op, int dim, int P) {
  if (P < kMinP || P > kMaxP || !op_has_tiles(op)) return 1;
  int c = 0;
  for (int k = 0; k < kMaxTiles; ++k)
    c += (dim == 3 ? kTileEPB3[P][k] : kTileEPB2[P][k]) > 0 ? 1 : 0;
  if (dim == 3 && op_has_lean(op)) {
    c *= kHelmForms;                       // each candidate also lean and deep
    if (packed_epb3(P) > 0) c += 1;        // and the packed slots
    if (helm_has_pt(P)) c *= 2;            // all again with the point-by-point I stage
  }
  return c;
}

// all candidates: the vector tiles, plus the matrix-core variant of the
// Helmholtz operator where it exists (always the last index)
int tile_count(int op, int dim, int P) {
  const int v = vector_tile_count(op, dim, P);
  if ((op == OP_HELM || op == OP_HELM_ASM) && mfma_supported(dim, P)) return v + 1;
  return v;
}

const char* tile_name(int op, int dim, int P, int tile) {
  static thread_local char buf[64];
  if (P < kMinP || P > kMaxP) return "";
  if ((op == OP_HELM || op == OP_HELM_ASM) && mfma_supported(dim, P) &&
      tile == vector_tile_count(op, dim, P)) {
    std::snprintf(buf, sizeof buf, "mfma_epb2_thr128");
    return buf;
  }
  const char* pt = "";
  if (dim == 3 && op_has_lean(op) && helm_has_pt(P)) {
    const int half = vector_tile_count(op, dim, P) / 2;
    if (tile >= half) {
      tile -= half;
      pt = "_pt";
    }
  }
  const int form = dim == 3 && op_has_lean(op) ? tile / epb3_count(P) : 0;   // 0, lean, deep
  const int q = P + 2;
  const int q2 = q * q;
  if (form == kHelmForms) {
    std::snprintf(buf, sizeof buf, "epb%d_thr%d_packed%s", packed_epb3(P), packed_epb3(P) * q2, pt);
    return buf;
  }
  if (dim == 3) tile %= epb3_count(P);
  const int epb = dim == 3 ? kTileEPB3[P][tile] : kTileEPB2[P][tile];
  const int slot = dim == 3 ? (q2 <= 16 ? 16 : q2 <= 64 ? 64 : q2) : q;
  std::snprintf(buf, sizeof buf, "epb%d_thr%d%s%s", epb, epb * slot,
                form == 1 ? "_lean" : form == 2 ? "_deep" : "", pt);
  return buf;
}

static int cur_tile(int op, int dim, int P, nk_dtype t) {
  if (op == OP_HELM_ASM) op = OP_HELM;
  if (!op_has_tiles(op) || P < kMinP || P > kMaxP) return 0;
  static std::once_flag once;
  std::call_once(once, [] {
    // NK_TILE forces one candidate index for every operator (testing aid)
    const char* f = std::getenv("NK_TILE");
    const int v = f ? std::atoi(f) : 0;
    for (auto& a : g_tile)
      for (auto& b : a)
        for (auto& c : b)
          for (auto& d : c) d.store(v);
    for (auto& a : g_tile_forced)
      for (auto& b : a)
        for (auto& c : b) c.store(f != nullptr);
  });
  int k = g_tile[op][dim - 2][P][t].load();
  if (k < 0 || k >= tile_count(op, dim, P)) k = 0;
  return k;
}

// ------------------------------------------------------------- validation
static nk_status check_device() {
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess || n <= 0)
    return fail(NK_EDEVICE, "no usable HIP device");
  return NK_OK;
}

// A device buffer argument must be GPU-accessible memory with at least
// `bytes` bytes from p to the end of its allocation.
static nk_status check_buf(const void* p, size_t bytes, const char* name) {
  if (bytes == 0) return NK_OK;
  if (p == nullptr) return fail(NK_EINVAL, std::string(name) + " is NULL");
  hipPointerAttribute_t attr;
  std::memset(&attr, 0, sizeof attr);
  if (hipPointerGetAttributes(&attr, p) != hipSuccess) {
    (void)hipGetLastError();
    return fail(NK_EINVAL, std::string(name) + " is not device memory");
  }
  if (attr.type != hipMemoryTypeDevice && attr.type != hipMemoryTypeManaged &&
      attr.type != hipMemoryTypeUnified) {
    return fail(NK_EINVAL, std::string(name) + " is not device memory");
  }
  hipDeviceptr_t base = nullptr;
  size_t size = 0;
  if (hipMemGetAddressRange(&base, &size, (hipDeviceptr_t)p) == hipSuccess && base != nullptr) {
    const size_t off = (const char*)p - (const char*)base;
    if (off + bytes > size)
      return fail(NK_EINVAL, std::string(name) + " is smaller than required (" +
                                 std::to_string(bytes) + " bytes)");
  } else {
    (void)hipGetLastError();
  }
  return NK_OK;
}

#define NK_CHECK(expr)               \
  do {                               \
    nk_status st_ = (expr);          \
    if (st_ != NK_OK) return st_;    \
  } while (0)

static size_t dsize(nk_dtype t) { return t == NK_F64 ? 8 : 4; }

static int64_t ipow(int64_t b, int e) {
  int64_t r = 1;
  for (int i = 0; i < e; ++i) r *= b;
  return r;
}

template <typename T>
static hipError_t dmalloc(T** p, size_t count) {
  *p = nullptr;
  if (count == 0) return hipSuccess;
  return hipMalloc((void**)p, count * sizeof(T));
}

template <typename T>
static void dfree(T*& p) {
  if (p) (void)hipFree(p);
  p = nullptr;
}

}  // namespace nk

using namespace nk;

// =================================================================== ABI
// The entry points below were declared extern "C" in nk.h, so their
// definitions have C linkage.

const char* nk_last_error(void) { return g_err.c_str(); }

int nk_version(void) { return 10000; }

int nk_device_count(void) {
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess) {
    (void)hipGetLastError();
    return 0;
  }
  return n;
}

nk_status nk_basis_tables(int P, int Q, double* x, double* w, double* B, double* DB) {
  if (P < 1 || Q < P + 1 || Q > 32) return fail(NK_EINVAL, "need 1 <= P, P+1 <= Q <= 32");
  std::vector<double> xx(Q), ww(Q), bb(Q * (P + 1)), dd(Q * (P + 1));
  gll_points(Q, xx.data(), ww.data());
  modified_basis(P, Q, xx.data(), bb.data(), dd.data());
  if (x) std::memcpy(x, xx.data(), Q * sizeof(double));
  if (w) std::memcpy(w, ww.data(), Q * sizeof(double));
  if (B) std::memcpy(B, bb.data(), bb.size() * sizeof(double));
  if (DB) std::memcpy(DB, dd.data(), dd.size() * sizeof(double));
  return NK_OK;
}

static void space_free(nk_space s) {
  if (!s) return;
  for (hipStream_t g : s->gstreams)
    if (g) (void)hipStreamDestroy(g);
  for (hipEvent_t g : s->gevents)
    if (g) (void)hipEventDestroy(g);
  if (s->fork) (void)hipEventDestroy(s->fork);
  dfree(s->fac64);
  dfree(s->fac32);
  dfree(s->dfac64);
  dfree(s->dfac32);
  dfree(s->kappa);
  dfree(s->varp_groups);
  dfree(s->varp_item_start);
  dfree(s->varp_lam_off);
  delete s;
}

nk_status nk_space_create_varp(nk_space* out, int dim, int ngroups, const int* P, const int* Q,
                               const int64_t* nelem, const double* const* jac,
                               const double* const* kappa, void* stream) {
  if (!out) return fail(NK_EINVAL, "out is NULL");
  *out = nullptr;
  if (dim != 2 && dim != 3) return fail(NK_EINVAL, "dim must be 2 or 3");
  if (ngroups < 1 || ngroups > 64) return fail(NK_EINVAL, "ngroups must be in [1, 64]");
  if (!P || !Q || !nelem || !jac) return fail(NK_EINVAL, "P, Q, nelem and jac must be non-NULL");
  for (int g = 0; g < ngroups; ++g) {
    if (nelem[g] < 0) return fail(NK_EINVAL, "nelem must be >= 0");
    if (nelem[g] > 0 && jac[g] == nullptr) return fail(NK_EINVAL, "jac is NULL");
    if (P[g] < 1 || Q[g] < P[g] + 1) return fail(NK_EINVAL, "need P >= 1 and Q >= P+1");
    if (!op_supported(dim, P[g], Q[g]))
      return fail(NK_EUNSUPPORTED, "compiled orders: 1 <= P <= 10 with Q = P + 2");
  }
  NK_CHECK(check_device());
  hipStream_t st = (hipStream_t)stream;
  nk_space s = new nk_space_s();
  s->dim = dim;
  (void)hipGetDevice(&s->device);
  bool has_kappa = false;
  for (int g = 0; g < ngroups; ++g) {
    Group G;
    G.P = P[g];
    G.Q = Q[g];
    G.n = P[g] + 1;
    G.nelem = nelem[g];
    G.e0 = s->nelem;
    G.c0 = s->ncoeff;
    G.q0 = s->npoint;
    G.f0 = s->nfac;
    G.d0 = s->ndfac;
    s->nelem += G.nelem;
    s->ncoeff += G.nelem * ipow(G.n, dim);
    s->npoint += G.nelem * ipow(G.Q, dim);
    s->nfac += G.nelem * ipow(G.Q, dim) * (dim == 3 ? kNF3 : kNF2);
    s->ndfac += G.nelem * ipow(G.Q, dim) * (dim * dim + 1);
    s->groups.push_back(G);
    if (kappa && kappa[g]) has_kappa = true;
  }
  for (int g = 0; g < ngroups; ++g) {
    const Group& G = s->groups[g];
    const int64_t nq = ipow(G.Q, dim);
    nk_status cs = check_buf(jac[g], (size_t)G.nelem * dim * dim * nq * 8, "jac");
    if (cs == NK_OK && kappa && kappa[g]) cs = check_buf(kappa[g], (size_t)G.nelem * nq * 8, "kappa");
    if (cs != NK_OK) {
      space_free(s);
      return cs;
    }
  }
  auto cleanup = [&](nk_status stt) {
    space_free(s);
    return stt;
  };
  hipError_t e;
  if ((e = dmalloc(&s->fac64, s->nfac)) != hipSuccess) return cleanup(hip_fail(e, "hipMalloc"));
  if ((e = dmalloc(&s->fac32, s->nfac)) != hipSuccess) return cleanup(hip_fail(e, "hipMalloc"));
  if ((e = dmalloc(&s->dfac64, s->ndfac)) != hipSuccess) return cleanup(hip_fail(e, "hipMalloc"));
  if ((e = dmalloc(&s->dfac32, s->ndfac)) != hipSuccess) return cleanup(hip_fail(e, "hipMalloc"));
  if (has_kappa) {
    if ((e = dmalloc(&s->kappa, s->npoint)) != hipSuccess) return cleanup(hip_fail(e, "hipMalloc"));
  }
  int* d_bad = nullptr;
  double* d_w = nullptr;
  if ((e = dmalloc(&d_bad, 1)) != hipSuccess) return cleanup(hip_fail(e, "hipMalloc"));
  if ((e = dmalloc(&d_w, 32)) != hipSuccess) {
    dfree(d_bad);
    return cleanup(hip_fail(e, "hipMalloc"));
  }
  e = hipMemsetAsync(d_bad, 0, sizeof(int), st);
  for (int g = 0; g < ngroups && e == hipSuccess; ++g) {
    const Group& G = s->groups[g];
    std::vector<double> x(G.Q), w(G.Q);
    gll_points(G.Q, x.data(), w.data());
    e = hipMemcpyAsync(d_w, w.data(), G.Q * sizeof(double), hipMemcpyHostToDevice, st);
    if (e != hipSuccess) break;
    const double* kg = (kappa && kappa[g]) ? kappa[g] : nullptr;
    if (has_kappa) {
      const int64_t nq = ipow(G.Q, dim);
      if (kg)
        e = hipMemcpyAsync(s->kappa + G.q0, kg, G.nelem * nq * sizeof(double),
                           hipMemcpyDeviceToDevice, st);
      else
        e = vec_fill<double>(s->kappa + G.q0, G.nelem * nq, 1.0, st);
      if (e != hipSuccess) break;
    }
    e = launch_geom(dim, G.Q, G.nelem, jac[g], kg, d_w, s->fac64 + G.f0, s->fac32 + G.f0,
                    s->dfac64 + G.d0, s->dfac32 + G.d0, d_bad, st);
    // the weights buffer is reused by the next group: wait for this launch
    if (e == hipSuccess) e = hipStreamSynchronize(st);
  }
  int bad = 0;
  if (e == hipSuccess) e = hipMemcpy(&bad, d_bad, sizeof(int), hipMemcpyDeviceToHost);
  dfree(d_bad);
  dfree(d_w);
  if (e != hipSuccess) return cleanup(hip_fail(e, "space setup"));
  if (bad) return cleanup(fail(NK_EINVAL, "non-positive Jacobian determinant or kappa"));
  if (ngroups > 1) {
    // persistent mixed-order launch tables: items of larger orders first
    std::vector<int> order(ngroups);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(),
                     [&](int a, int b) { return s->groups[a].P > s->groups[b].P; });
    std::vector<VarpGroup> vg;
    std::vector<int64_t> start(1, 0), lamoff;
    for (int k : order) {
      const Group& G = s->groups[k];
      VarpGroup v;
      v.P = G.P;
      v.nelem = G.nelem;
      v.c0 = G.c0;
      v.f0 = G.f0;
      vg.push_back(v);
      lamoff.push_back(G.e0);
      start.push_back(start.back() + varp_items_per_group(G.P, G.nelem));
    }
    s->varp_nitems = start.back();
    if ((e = dmalloc(&s->varp_groups, vg.size())) != hipSuccess ||
        (e = dmalloc(&s->varp_item_start, start.size())) != hipSuccess ||
        (e = dmalloc(&s->varp_lam_off, lamoff.size())) != hipSuccess)
      return cleanup(hip_fail(e, "hipMalloc"));
    e = hipMemcpy(s->varp_groups, vg.data(), vg.size() * sizeof(VarpGroup), hipMemcpyHostToDevice);
    if (e == hipSuccess)
      e = hipMemcpy(s->varp_item_start, start.data(), start.size() * 8, hipMemcpyHostToDevice);
    if (e == hipSuccess)
      e = hipMemcpy(s->varp_lam_off, lamoff.data(), lamoff.size() * 8, hipMemcpyHostToDevice);
    if (e != hipSuccess) return cleanup(hip_fail(e, "hipMemcpy"));
  }
  *out = s;
  return NK_OK;
}

nk_status nk_space_create(nk_space* out, int dim, int64_t nelem, int P, int Q, const double* jac,
                          const double* kappa, void* stream) {
  const double* j[1] = {jac};
  const double* k[1] = {kappa};
  return nk_space_create_varp(out, dim, 1, &P, &Q, &nelem, j, kappa ? k : nullptr, stream);
}

nk_status nk_tri_points(int Q, double* eta1, double* w1, double* eta2, double* w2) {
  if (Q < 3 || Q > kMaxP + 2 || !eta1 || !w1 || !eta2 || !w2)
    return fail(NK_EINVAL, "need 3 <= Q <= 12 and non-NULL outputs");
  tri_points(Q, eta1, w1, eta2, w2);
  return NK_OK;
}

nk_status nk_space_create_tri(nk_space* out, int64_t nelem, int P, int Q, const double* jac,
                              const double* kappa, void* stream) {
  if (!out) return fail(NK_EINVAL, "out is NULL");
  *out = nullptr;
  if (nelem < 0) return fail(NK_EINVAL, "nelem must be >= 0");
  if (P < 1 || P > kMaxP || Q != P + 2)
    return fail(NK_EUNSUPPORTED, "compiled triangle orders: 1 <= P <= 10 with Q = P + 2");
  const int64_t NP = (int64_t)Q * (Q - 1), NM = (int64_t)(P + 1) * (P + 2) / 2;
  if (nelem > 0 && !jac) return fail(NK_EINVAL, "jac is NULL");
  NK_CHECK(check_buf(jac, (size_t)nelem * 4 * NP * 8, "jac"));
  if (kappa) NK_CHECK(check_buf(kappa, (size_t)nelem * NP * 8, "kappa"));
  NK_CHECK(check_device());
  hipStream_t st = (hipStream_t)stream;
  nk_space s = new nk_space_s();
  s->dim = 2;
  s->shape = 1;
  (void)hipGetDevice(&s->device);
  Group G;
  G.P = P;
  G.Q = Q;
  G.n = P + 1;
  G.nelem = nelem;
  s->groups.push_back(G);
  s->nelem = nelem;
  s->ncoeff = nelem * NM;
  s->npoint = nelem * NP;
  s->nfac = tri_fac_count(Q, nelem);   // padded to whole wavefront groups
  auto cleanup = [&](nk_status stt) {
    space_free(s);
    return stt;
  };
  hipError_t e;
  if ((e = dmalloc(&s->fac64, s->nfac)) || (e = dmalloc(&s->fac32, s->nfac)))
    return cleanup(hip_fail(e, "hipMalloc"));
  std::vector<double> pts(2 * Q + 2 * (Q - 1));
  tri_points(Q, pts.data(), pts.data() + Q, pts.data() + 2 * Q, pts.data() + 2 * Q + (Q - 1));
  int* d_bad = nullptr;
  double* d_pts = nullptr;
  if ((e = dmalloc(&d_bad, 1)) || (e = dmalloc(&d_pts, pts.size()))) {
    dfree(d_bad);
    return cleanup(hip_fail(e, "hipMalloc"));
  }
  int bad = 0;
  if (!(e = hipMemsetAsync(d_bad, 0, sizeof(int), st)) &&
      !(e = hipMemsetAsync(s->fac64, 0, s->nfac * 8, st)) &&
      !(e = hipMemsetAsync(s->fac32, 0, s->nfac * 4, st)) &&
      !(e = hipMemcpyAsync(d_pts, pts.data(), pts.size() * 8, hipMemcpyHostToDevice, st)) &&
      !(e = launch_geom_tri(Q, nelem, jac, kappa, d_pts, s->fac64, s->fac32, d_bad, st)) &&
      !(e = hipStreamSynchronize(st)))
    e = hipMemcpy(&bad, d_bad, sizeof(int), hipMemcpyDeviceToHost);
  dfree(d_bad);
  dfree(d_pts);
  if (e != hipSuccess) return cleanup(hip_fail(e, "triangle space setup"));
  if (bad) return cleanup(fail(NK_EINVAL, "non-positive Jacobian determinant or kappa"));
  *out = s;
  return NK_OK;
}

nk_status nk_tet_points(int Q, double* eta1, double* w1, double* eta2, double* w2, double* eta3,
                        double* w3) {
  if (Q < 3 || Q > kMaxP + 2 || !eta1 || !w1 || !eta2 || !w2 || !eta3 || !w3)
    return fail(NK_EINVAL, "need 3 <= Q <= 12 and non-NULL outputs");
  tet_points(Q, eta1, w1, eta2, w2, eta3, w3);
  return NK_OK;
}

// Tetrahedra (shape 2), prisms (shape 3) and pyramids (shape 4): one order
// group, 7 factors per point built by the collapsed-shape geometry kernel.
static nk_status space_create_col3(nk_space* out, int shape, int64_t nelem, int P, int Q,
                                   const double* jac, const double* kappa, void* stream) {
  if (!out) return fail(NK_EINVAL, "out is NULL");
  *out = nullptr;
  if (nelem < 0) return fail(NK_EINVAL, "nelem must be >= 0");
  if (P < 1 || P > kMaxP || Q != P + 2)
    return fail(NK_EUNSUPPORTED, "compiled orders: 1 <= P <= 10 with Q = P + 2");
  const bool tet = shape == 2, pyr = shape == 4;
  const int Q2 = pyr ? Q : Q - 1, Q3 = shape == 3 ? Q : Q - 1;
  const int64_t NP = (int64_t)Q * Q2 * Q3;
  const int64_t NM = tet   ? (int64_t)(P + 1) * (P + 2) * (P + 3) / 6
                     : pyr ? (int64_t)(P + 1) * (P + 2) * (2 * P + 3) / 6
                           : (int64_t)(P + 1) * (P + 1) * (P + 2) / 2;
  if (nelem > 0 && !jac) return fail(NK_EINVAL, "jac is NULL");
  NK_CHECK(check_buf(jac, (size_t)nelem * 9 * NP * 8, "jac"));
  if (kappa) NK_CHECK(check_buf(kappa, (size_t)nelem * NP * 8, "kappa"));
  NK_CHECK(check_device());
  hipStream_t st = (hipStream_t)stream;
  nk_space s = new nk_space_s();
  s->dim = 3;
  s->shape = shape;
  (void)hipGetDevice(&s->device);
  Group G;
  G.P = P;
  G.Q = Q;
  G.n = P + 1;
  G.nelem = nelem;
  s->groups.push_back(G);
  s->nelem = nelem;
  s->ncoeff = nelem * NM;
  s->npoint = nelem * NP;
  s->nfac = nelem * 7 * NP;
  auto cleanup = [&](nk_status stt) {
    space_free(s);
    return stt;
  };
  hipError_t e;
  if ((e = dmalloc(&s->fac64, s->nfac)) || (e = dmalloc(&s->fac32, s->nfac)))
    return cleanup(hip_fail(e, "hipMalloc"));
  // e1, w1 (Q), e2, w2 (Q2), e3, w3 (Q3)
  std::vector<double> pts(2 * Q + 2 * Q2 + 2 * Q3);
  double* p = pts.data();
  double* p3 = p + 2 * Q + 2 * Q2;
  if (tet) {
    tet_points(Q, p, p + Q, p + 2 * Q, p + 2 * Q + Q2, p3, p3 + Q3);
  } else if (pyr) {
    gll_points(Q, p, p + Q);
    gll_points(Q, p + 2 * Q, p + 3 * Q);
    radau_points(Q3, 2, p3, p3 + Q3);
  } else {
    tri_points(Q, p, p + Q, p + 2 * Q, p + 2 * Q + Q2);
    gll_points(Q, p3, p3 + Q3);
  }
  int* d_bad = nullptr;
  double* d_pts = nullptr;
  if ((e = dmalloc(&d_bad, 1)) || (e = dmalloc(&d_pts, pts.size()))) {
    dfree(d_bad);
    return cleanup(hip_fail(e, "hipMalloc"));
  }
  int bad = 0;
  if (!(e = hipMemsetAsync(d_bad, 0, sizeof(int), st)) &&
      !(e = hipMemcpyAsync(d_pts, pts.data(), pts.size() * 8, hipMemcpyHostToDevice, st)) &&
      !(e = tet   ? launch_geom_tet(Q, nelem, jac, kappa, d_pts, s->fac64, s->fac32, d_bad, st)
            : pyr ? launch_geom_pyr(Q, nelem, jac, kappa, d_pts, s->fac64, s->fac32, d_bad, st)
                  : launch_geom_prism(Q, nelem, jac, kappa, d_pts, s->fac64, s->fac32, d_bad, st)) &&
      !(e = hipStreamSynchronize(st)))
    e = hipMemcpy(&bad, d_bad, sizeof(int), hipMemcpyDeviceToHost);
  dfree(d_bad);
  dfree(d_pts);
  if (e != hipSuccess) return cleanup(hip_fail(e, "collapsed-shape space setup"));
  if (bad) return cleanup(fail(NK_EINVAL, "non-positive Jacobian determinant or kappa"));
  *out = s;
  return NK_OK;
}

nk_status nk_space_create_tet(nk_space* out, int64_t nelem, int P, int Q, const double* jac,
                              const double* kappa, void* stream) {
  return space_create_col3(out, 2, nelem, P, Q, jac, kappa, stream);
}

nk_status nk_space_create_prism(nk_space* out, int64_t nelem, int P, int Q, const double* jac,
                                const double* kappa, void* stream) {
  return space_create_col3(out, 3, nelem, P, Q, jac, kappa, stream);
}

nk_status nk_space_create_pyr(nk_space* out, int64_t nelem, int P, int Q, const double* jac,
                              const double* kappa, void* stream) {
  return space_create_col3(out, 4, nelem, P, Q, jac, kappa, stream);
}

nk_status nk_space_destroy(nk_space s) {
  if (!s) return fail(NK_EINVAL, "space is NULL");
  (void)hipDeviceSynchronize();
  space_free(s);
  return NK_OK;
}

nk_status nk_space_sizes(nk_space s, int64_t* nelem, int64_t* ncoeffs, int64_t* npoints) {
  if (!s) return fail(NK_EINVAL, "space is NULL");
  if (nelem) *nelem = s->nelem;
  if (ncoeffs) *ncoeffs = s->ncoeff;
  if (npoints) *npoints = s->npoint;
  return NK_OK;
}

// Run one elemental operator over every group of the space.
static nk_status space_op(nk_space s, int op, nk_dtype t, const void* in, void* out,
                          const double* lam, double lam0, const double* in2, void* stream) {
  if (!s) return fail(NK_EINVAL, "space is NULL");
  if (t != NK_F64 && t != NK_F32) return fail(NK_EINVAL, "bad dtype");
  const size_t sz = dsize(t);
  const int d = s->dim;
  const bool pts_in = (op == OP_IPROD || op == OP_RHS);
  const bool pts_out = (op == OP_BWD);
  NK_CHECK(check_buf(in, (pts_in ? s->npoint : s->ncoeff) * sz, "input"));
  NK_CHECK(check_buf(out, (pts_out ? s->npoint : s->ncoeff) * sz, "output"));
  if (lam) NK_CHECK(check_buf(lam, s->nelem * 8, "lambda"));
  if (op == OP_RHS) NK_CHECK(check_buf(in2, s->npoint * d * 8, "du"));
  if (in == out && in != nullptr) return fail(NK_EINVAL, "input and output must not alias");
  if (s->shape != 0 && op != OP_BWD && op != OP_IPROD && op != OP_HELM)
    return fail(NK_EUNSUPPORTED, "collapsed-coordinate spaces provide BwdTrans, IProductWRTBase and Helmholtz");
  hipStream_t st = (hipStream_t)stream;
  const char* fac = t == NK_F64 ? (const char*)s->fac64 : (const char*)s->fac32;
  auto group_args = [&](const Group& G) {
    OpArgs a;
    a.op = op;
    a.dim = d;
    a.P = G.P;
    a.Q = G.Q;
    a.nelem = G.nelem;
    a.in = (const char*)in + (pts_in ? G.q0 : G.c0) * sz;
    a.out = (char*)out + (pts_out ? G.q0 : G.c0) * sz;
    a.fac = fac + G.f0 * sz;
    a.lam = lam ? lam + G.e0 : nullptr;
    a.lam0 = lam0;
    a.in2 = in2 ? in2 + G.q0 * d : nullptr;
    a.tile = cur_tile(op, d, G.P, t);
    a.stream = st;
    return a;
  };
  if (s->shape == 1) {
    const hipError_t e = launch_tri(t, group_args(s->groups[0]));
    if (e != hipSuccess) return hip_fail(e, "triangle operator launch");
    return NK_OK;
  }
  if (s->shape >= 2) {
    const hipError_t e = s->shape == 2   ? launch_tet(t, group_args(s->groups[0]))
                         : s->shape == 3 ? launch_prism(t, group_args(s->groups[0]))
                                         : launch_pyr(t, group_args(s->groups[0]));
    if (e != hipSuccess) return hip_fail(e, "collapsed-shape operator launch");
    return NK_OK;
  }
  int strategy = VARP_SEQUENTIAL;
  if (s->groups.size() > 1)
    strategy = (op == OP_HELM) ? s->varp_strategy[t] : VARP_CONCURRENT;
  if (strategy == VARP_PERSISTENT || strategy == VARP_PERSISTENT_2) {
    VarpArgs v;
    v.t = t;
    v.ngroups = (int)s->groups.size();
    v.groups_dev = s->varp_groups;
    v.item_start_dev = s->varp_item_start;
    v.nitems = s->varp_nitems;
    v.x = in;
    v.y = out;
    v.fac = fac;
    v.lam = lam;
    v.lam_off_dev = s->varp_lam_off;
    v.lam0 = lam0;
    v.minb = strategy == VARP_PERSISTENT_2 ? 2 : 1;
    int ncu = 0;
    (void)hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, s->device);
    const int64_t grid = std::min<int64_t>(
        (int64_t)std::max(ncu, 1) * varp_blocks_per_cu(t, v.minb), s->varp_nitems);
    v.grid = (int)std::max<int64_t>(grid, 1);
    v.stream = st;
    hipError_t e = launch_helm_varp(v);
    if (e != hipSuccess) return hip_fail(e, "mixed-order Helmholtz launch");
    return NK_OK;
  }
  if (strategy == VARP_CONCURRENT) {
    // fork/join: every order group on its own stream, all ordered after the
    // caller's work and joined back into the caller's stream
    hipError_t e = hipSuccess;
    if (s->gstreams.empty()) {
      for (size_t g = 0; g < s->groups.size() && e == hipSuccess; ++g) {
        hipStream_t gs = nullptr;
        hipEvent_t ge = nullptr;
        e = hipStreamCreateWithFlags(&gs, hipStreamNonBlocking);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&ge, hipEventDisableTiming);
        s->gstreams.push_back(gs);
        s->gevents.push_back(ge);
      }
      if (e == hipSuccess) e = hipEventCreateWithFlags(&s->fork, hipEventDisableTiming);
      if (e != hipSuccess) return hip_fail(e, "stream creation");
    }
    if ((e = hipEventRecord(s->fork, st))) return hip_fail(e, "hipEventRecord");
    for (size_t g = 0; g < s->groups.size(); ++g) {
      OpArgs a = group_args(s->groups[g]);
      a.stream = s->gstreams[g];
      if ((e = hipStreamWaitEvent(a.stream, s->fork, 0))) return hip_fail(e, "hipStreamWaitEvent");
      if ((e = launch_op(d, t, a))) return hip_fail(e, "operator launch");
      if ((e = hipEventRecord(s->gevents[g], a.stream))) return hip_fail(e, "hipEventRecord");
    }
    for (size_t g = 0; g < s->groups.size(); ++g)
      if ((e = hipStreamWaitEvent(st, s->gevents[g], 0))) return hip_fail(e, "hipStreamWaitEvent");
    return NK_OK;
  }
  for (const Group& G : s->groups) {
    hipError_t e = launch_op(d, t, group_args(G));
    if (e != hipSuccess) return hip_fail(e, "operator launch");
  }
  return NK_OK;
}

nk_status nk_space_set_strategy(nk_space s, nk_dtype t, int strategy) {
  if (!s) return fail(NK_EINVAL, "space is NULL");
  if (t != NK_F64 && t != NK_F32) return fail(NK_EINVAL, "bad dtype");
  if (strategy < 0 || strategy >= VARP_COUNT) return fail(NK_EINVAL, "bad strategy");
  s->varp_strategy[t] = strategy;
  return NK_OK;
}

int nk_space_get_strategy(nk_space s, nk_dtype t) {
  if (!s || (t != NK_F64 && t != NK_F32)) return -1;
  return s->varp_strategy[t];
}

nk_status nk_bwd_trans(nk_space s, nk_dtype t, const void* coeffs, void* phys, void* stream) {
  return space_op(s, OP_BWD, t, coeffs, phys, nullptr, 0.0, nullptr, stream);
}

nk_status nk_iprod_wrt_base(nk_space s, nk_dtype t, const void* phys, void* coeffs, void* stream) {
  return space_op(s, OP_IPROD, t, phys, coeffs, nullptr, 0.0, nullptr, stream);
}

nk_status nk_helmholtz(nk_space s, nk_dtype t, const double* lambda, double lambda0, const void* x,
                       void* y, void* stream) {
  return space_op(s, OP_HELM, t, x, y, lambda, lambda0, nullptr, stream);
}

nk_status nk_helmholtz_weak_rhs(nk_space s, const double* lambda, double lambda0, const double* u,
                                const double* du, double* y, void* stream) {
  return space_op(s, OP_RHS, NK_F64, u, y, lambda, lambda0, du, stream);
}

// PhysDeriv, IProductWRTDerivBase and FwdTrans: one launch per order group.
static nk_status deriv_op(nk_space s, int which, nk_dtype t, const void* in, void* out,
                          void* stream) {
  if (!s) return fail(NK_EINVAL, "space is NULL");
  if (t != NK_F64 && t != NK_F32) return fail(NK_EINVAL, "bad dtype");
  const size_t sz = dsize(t);
  const int d = s->dim;
  if (s->shape != 0) return fail(NK_EUNSUPPORTED, "derivative operators are built for quadrilaterals and hexahedra");
  // element-major blocks: points [Q^d], vector fields [d][Q^d], coefficients [n^d]
  const int64_t vin = which == DERIV_IPROD ? d : 1, vout = which == DERIV_PHYS ? d : 1;
  const bool coeff_out = which != DERIV_PHYS;
  NK_CHECK(check_buf(in, s->npoint * vin * sz, "input"));
  NK_CHECK(check_buf(out, (coeff_out ? s->ncoeff : s->npoint * vout) * sz, "output"));
  if (in == out && in != nullptr) return fail(NK_EINVAL, "input and output must not alias");
  const char* df = t == NK_F64 ? (const char*)s->dfac64 : (const char*)s->dfac32;
  for (const Group& G : s->groups) {
    DerivArgs a;
    a.nelem = G.nelem;
    a.in = (const char*)in + G.q0 * vin * sz;
    a.out = (char*)out + (coeff_out ? G.c0 : G.q0 * vout) * sz;
    a.dfac = df + G.d0 * sz;
    a.stream = (hipStream_t)stream;
    const hipError_t e = launch_deriv(t, which, d, G.P, a);
    if (e != hipSuccess) return hip_fail(e, "derivative operator launch");
  }
  return NK_OK;
}

nk_status nk_phys_deriv(nk_space s, nk_dtype t, const void* phys, void* deriv, void* stream) {
  return deriv_op(s, DERIV_PHYS, t, phys, deriv, stream);
}

nk_status nk_iprod_wrt_deriv_base(nk_space s, nk_dtype t, const void* f, void* coeffs,
                                  void* stream) {
  return deriv_op(s, DERIV_IPROD, t, f, coeffs, stream);
}

nk_status nk_fwd_trans(nk_space s, nk_dtype t, const void* phys, void* coeffs, void* stream) {
  return deriv_op(s, DERIV_FWD, t, phys, coeffs, stream);
}

nk_status nk_helmholtz_param_grad(nk_space s, const double* z_loc, const double* u_loc,
                                  double* dkappa, double* dlambda, void* stream) {
  if (!s) return fail(NK_EINVAL, "space is NULL");
  if (s->groups.size() != 1) return fail(NK_EINVAL, "gradient needs a single-order space");
  if (s->shape != 0) return fail(NK_EUNSUPPORTED, "gradient kernel is built for hexahedra");
  NK_CHECK(check_buf(z_loc, s->ncoeff * 8, "z_loc"));
  NK_CHECK(check_buf(u_loc, s->ncoeff * 8, "u_loc"));
  if (dkappa) NK_CHECK(check_buf(dkappa, s->npoint * 8, "dkappa"));
  if (dlambda) NK_CHECK(check_buf(dlambda, s->nelem * 8, "dlambda"));
  const Group& G = s->groups[0];
  OpArgs a;
  a.op = OP_GRAD;
  a.dim = s->dim;
  a.P = G.P;
  a.Q = G.Q;
  a.nelem = G.nelem;
  a.in = z_loc;
  a.in2 = u_loc;
  a.out = dkappa;
  a.out2 = dlambda;
  a.fac = s->fac64;
  a.kappa = s->kappa;
  a.stream = (hipStream_t)stream;
  hipError_t e = launch_op(s->dim, NK_F64, a);
  if (e != hipSuccess) return hip_fail(e, "gradient launch");
  return NK_OK;
}

// ================================================================ systems
static void cond_free(CondData*& c);

static void system_free(nk_system y) {
  if (!y) return;
  if (y->cs) (void)hipStreamSynchronize(y->cs);
  cond_free(y->cond);
  if (y->g64) (void)hipGraphExecDestroy(y->g64);
  if (y->g32) (void)hipGraphExecDestroy(y->g32);
  dfree(y->d_dof_off);
  dfree(y->d_pdof_off);
  dfree(y->d_elem_off);
  dfree(y->d_blk_first);
  dfree(y->d_blk_seg);
  dfree(y->dslot);
  dfree(y->elem_seg);
  dfree(y->l2g);
  dfree(y->lam);
  dfree(y->diag);
  dfree(y->dinv64);
  dfree(y->dinv32);
  dfree(y->b);
  dfree(y->x);
  dfree(y->r);
  dfree(y->p);
  dfree(y->y);
  dfree(y->u);
  dfree(y->s);
  dfree(y->u32);
  dfree(y->s32);
  dfree(y->r32);
  dfree(y->p32);
  dfree(y->y32);
  dfree(y->d32);
  dfree(y->part);
  for (CgState* c : {&y->st64, &y->st32}) {
    dfree(c->rz);
    dfree(c->rr);
    dfree(c->tol2);
    dfree(c->alpha);
    dfree(c->done);
    dfree(c->iters);
    dfree(c->status);
    dfree(c->cnt);
    dfree(c->maxit);
    dfree(c->gsl);
    dfree(c->dsl);
    dfree(c->sgam);
    dfree(c->salp);
    dfree(c->sit);
    dfree(c->sdn);
  }
  dfree(y->bb);
  dfree(y->rr_true);
  dfree(y->cnt_aux);
  dfree(y->outer_done);
  dfree(y->outer_tol2);
  dfree(y->outer_rr);
  dfree(y->outer_cnt);
  dfree(y->outer_status);
  if (y->h_flags) (void)hipHostFree(y->h_flags);
  if (y->h_budget) (void)hipHostFree(y->h_budget);
  if (y->h_d) (void)hipHostFree(y->h_d);
  if (y->ev) (void)hipEventDestroy(y->ev);
  for (hipStream_t gs : y->ostreams)
    if (gs) (void)hipStreamDestroy(gs);
  for (hipEvent_t ge : y->oevents)
    if (ge) (void)hipEventDestroy(ge);
  if (y->ofork) (void)hipEventDestroy(y->ofork);
  if (y->cs) (void)hipStreamDestroy(y->cs);
  delete y;
}

static hipError_t alloc_state(CgState& c, int n) {
  hipError_t e;
  if ((e = dmalloc(&c.rz, n)) || (e = dmalloc(&c.rr, n)) || (e = dmalloc(&c.tol2, n)) ||
      (e = dmalloc(&c.alpha, n)) || (e = dmalloc(&c.done, n)) || (e = dmalloc(&c.iters, n)) ||
      (e = dmalloc(&c.status, n)) || (e = dmalloc(&c.cnt, n)) || (e = dmalloc(&c.maxit, n)) ||
      (e = dmalloc(&c.gsl, (int64_t)3 * n * 2 * kSlots)) ||
      (e = dmalloc(&c.dsl, (int64_t)2 * n * kSlots)) || (e = dmalloc(&c.sgam, 2 * n)) ||
      (e = dmalloc(&c.salp, 2 * n)) || (e = dmalloc(&c.sit, 2 * n)) || (e = dmalloc(&c.sdn, 2 * n)))
    return e;
  return hipMemset(c.cnt, 0, n * sizeof(int32_t));
}

static int tune_asm_tile(nk_system y, nk_dtype t, int g, hipStream_t st);

static nk_status system_create(nk_system* out, nk_space s, int nsys, const int64_t* elem_off,
                               const int64_t* dof_off, const int32_t* l2g, const int8_t* sign,
                               const uint8_t* dirichlet, const double* lambda, double lambda0,
                               void* stream, bool tune = true) {
  if (!out) return fail(NK_EINVAL, "out is NULL");
  *out = nullptr;
  if (!s) return fail(NK_EINVAL, "space is NULL");
  if (nsys < 1) return fail(NK_EINVAL, "nsys must be >= 1");
  if (s->groups.size() != 1 && nsys != 1)
    return fail(NK_EINVAL, "a mixed-order space takes one system (nsys = 1)");
  if (s->shape != 0 && nsys != 1)
    return fail(NK_EINVAL, "a triangle, tetrahedron, prism or pyramid space takes one system (nsys = 1)");
  if (!elem_off || !dof_off) return fail(NK_EINVAL, "offsets must be non-NULL");
  if (elem_off[0] != 0 || elem_off[nsys] != s->nelem)
    return fail(NK_EINVAL, "elem_off must start at 0 and end at the space's element count");
  if (dof_off[0] != 0) return fail(NK_EINVAL, "dof_off must start at 0");
  for (int k = 0; k < nsys; ++k) {
    if (elem_off[k + 1] < elem_off[k] || dof_off[k + 1] < dof_off[k])
      return fail(NK_EINVAL, "offsets must be non-decreasing");
  }
  if (dof_off[nsys] >= ((int64_t)1 << 30)) return fail(NK_EINVAL, "too many global DOFs");
  if (s->ncoeff >= ((int64_t)1 << 31) - 1) return fail(NK_EINVAL, "too many local coefficients");
  NK_CHECK(check_buf(l2g, (size_t)s->ncoeff * 4, "l2g"));
  if (sign) NK_CHECK(check_buf(sign, (size_t)s->ncoeff, "sign"));
  NK_CHECK(check_buf(dirichlet, (size_t)dof_off[nsys], "dirichlet"));
  if (lambda) NK_CHECK(check_buf(lambda, s->nelem * 8, "lambda"));
  NK_CHECK(check_device());
  hipStream_t st = (hipStream_t)stream;
  nk_system y = new nk_system_s();
  y->space = s;
  y->nsys = nsys;
  y->lam0 = lambda0;
  (void)hipGetDevice(&y->device);
  y->dof_off.assign(dof_off, dof_off + nsys + 1);
  y->elem_off.assign(elem_off, elem_off + nsys + 1);
  y->nuser = dof_off[nsys];
  y->pdof_off.assign(nsys + 1, 0);
  y->blk_first.assign(nsys + 1, 0);
  for (int k = 0; k < nsys; ++k) {
    const int64_t nd = std::max<int64_t>(dof_off[k + 1] - dof_off[k], 1);
    const int64_t padded = (nd + kSegAlign - 1) / kSegAlign * kSegAlign;
    y->pdof_off[k + 1] = y->pdof_off[k] + padded;
    y->blk_first[k + 1] = y->pdof_off[k + 1] / kSegAlign;
  }
  y->L.npad = y->pdof_off[nsys];
  y->L.nblk = y->L.npad / kSegAlign;
  if (y->L.npad >= (int64_t)kL2gNeg) {   // bit 30 of an internal l2g entry is the sign flag
    system_free(y);
    return fail(NK_EINVAL, "padded system too large");
  }
  std::vector<int32_t> blk_seg(y->L.nblk), eseg(s->nelem), dslot(s->nelem);
  for (int k = 0; k < nsys; ++k) {
    for (int64_t b = y->blk_first[k]; b < y->blk_first[k + 1]; ++b) blk_seg[b] = k;
    for (int64_t e = elem_off[k]; e < elem_off[k + 1]; ++e) {
      eseg[e] = k;
      dslot[e] = (int32_t)(k * kSlots + (e - elem_off[k]) % kSlots);   // CG accumulation slot
    }
  }
  auto cleanup = [&](nk_status stt) {
    system_free(y);
    return stt;
  };
  hipError_t e = hipSuccess;
  const int64_t np = y->L.npad;
#define NK_ALLOC(ptr, n) \
  if ((e = dmalloc(&(ptr), (n))) != hipSuccess) return cleanup(hip_fail(e, "hipMalloc"))
  NK_ALLOC(y->d_dof_off, nsys + 1);
  NK_ALLOC(y->d_pdof_off, nsys + 1);
  NK_ALLOC(y->d_elem_off, nsys + 1);
  NK_ALLOC(y->d_blk_first, nsys + 1);
  NK_ALLOC(y->d_blk_seg, y->L.nblk);
  NK_ALLOC(y->elem_seg, std::max<int64_t>(s->nelem, 1));
  NK_ALLOC(y->l2g, std::max<int64_t>(s->ncoeff, 1));
  if (lambda) NK_ALLOC(y->lam, s->nelem);
  NK_ALLOC(y->diag, np);
  NK_ALLOC(y->dinv64, np);
  NK_ALLOC(y->dinv32, np);
  NK_ALLOC(y->b, np);
  NK_ALLOC(y->x, np);
  NK_ALLOC(y->r, np);
  NK_ALLOC(y->p, np);
  NK_ALLOC(y->y, np);
  NK_ALLOC(y->u, np);
  NK_ALLOC(y->s, np);
  NK_ALLOC(y->u32, np);
  NK_ALLOC(y->s32, np);
  NK_ALLOC(y->r32, np);
  NK_ALLOC(y->p32, np);
  NK_ALLOC(y->y32, np);
  NK_ALLOC(y->d32, np);
  NK_ALLOC(y->part, 2 * y->L.nblk);
  NK_ALLOC(y->dslot, std::max<int64_t>(s->nelem, 1));
  NK_ALLOC(y->bb, nsys);
  NK_ALLOC(y->rr_true, nsys);
  NK_ALLOC(y->cnt_aux, nsys);
  NK_ALLOC(y->outer_done, nsys);
  NK_ALLOC(y->outer_tol2, nsys);
  NK_ALLOC(y->outer_rr, nsys);
  NK_ALLOC(y->outer_cnt, nsys);
  NK_ALLOC(y->outer_status, nsys);
#undef NK_ALLOC
  if ((e = alloc_state(y->st64, nsys)) != hipSuccess) return cleanup(hip_fail(e, "hipMalloc"));
  if ((e = alloc_state(y->st32, nsys)) != hipSuccess) return cleanup(hip_fail(e, "hipMalloc"));
  if ((e = hipHostMalloc((void**)&y->h_flags, 2 * nsys * sizeof(int32_t), 0)) != hipSuccess)
    return cleanup(hip_fail(e, "hipHostMalloc"));
  if ((e = hipHostMalloc((void**)&y->h_budget, nsys * sizeof(int32_t), 0)) != hipSuccess)
    return cleanup(hip_fail(e, "hipHostMalloc"));
  if ((e = hipHostMalloc((void**)&y->h_d, nsys * sizeof(double), 0)) != hipSuccess)
    return cleanup(hip_fail(e, "hipHostMalloc"));
  if ((e = hipStreamCreateWithFlags(&y->cs, hipStreamNonBlocking)) != hipSuccess)
    return cleanup(hip_fail(e, "hipStreamCreate"));
  if ((e = hipEventCreateWithFlags(&y->ev, hipEventDisableTiming)) != hipSuccess)
    return cleanup(hip_fail(e, "hipEventCreate"));
  if (s->groups.size() > 1 && s->shape == 0) {   // side streams of the order groups (sys_op)
    for (size_t g = 1; g < s->groups.size(); ++g) {
      hipStream_t gs = nullptr;
      hipEvent_t ge = nullptr;
      if ((e = hipStreamCreateWithFlags(&gs, hipStreamNonBlocking)) != hipSuccess)
        return cleanup(hip_fail(e, "hipStreamCreate"));
      y->ostreams.push_back(gs);
      if ((e = hipEventCreateWithFlags(&ge, hipEventDisableTiming)) != hipSuccess)
        return cleanup(hip_fail(e, "hipEventCreate"));
      y->oevents.push_back(ge);
    }
    if ((e = hipEventCreateWithFlags(&y->ofork, hipEventDisableTiming)) != hipSuccess)
      return cleanup(hip_fail(e, "hipEventCreate"));
  }
  y->L.blk_seg = y->d_blk_seg;
  y->L.blk_first = y->d_blk_first;
  // setup runs on the caller's stream, then synchronises it
  int* d_bad = nullptr;
  double *d_B = nullptr, *d_D = nullptr;
  // 1-D tables of every order group, one after the other
  std::vector<double> hB, hD;
  std::vector<int64_t> tab_off;
  for (const Group& G : s->groups) {
    const int QN = G.Q * G.n;
    std::vector<double> xq(G.Q), wq(G.Q), b(QN), d(QN);
    gll_points(G.Q, xq.data(), wq.data());
    modified_basis(G.P, G.Q, xq.data(), b.data(), d.data());
    tab_off.push_back((int64_t)hB.size());
    hB.insert(hB.end(), b.begin(), b.end());
    hD.insert(hD.end(), d.begin(), d.end());
  }
  if ((e = dmalloc(&d_bad, 1)) || (e = dmalloc(&d_B, hB.size())) || (e = dmalloc(&d_D, hD.size()))) {
    dfree(d_bad);
    dfree(d_B);
    dfree(d_D);
    return cleanup(hip_fail(e, "hipMalloc"));
  }
  do {
    if ((e = hipMemcpyAsync(y->d_dof_off, dof_off, (nsys + 1) * 8, hipMemcpyHostToDevice, st))) break;
    if ((e = hipMemcpyAsync(y->d_pdof_off, y->pdof_off.data(), (nsys + 1) * 8, hipMemcpyHostToDevice, st))) break;
    if ((e = hipMemcpyAsync(y->d_elem_off, elem_off, (nsys + 1) * 8, hipMemcpyHostToDevice, st))) break;
    if ((e = hipMemcpyAsync(y->d_blk_first, y->blk_first.data(), (nsys + 1) * 8, hipMemcpyHostToDevice, st))) break;
    if ((e = hipMemcpyAsync(y->d_blk_seg, blk_seg.data(), y->L.nblk * 4, hipMemcpyHostToDevice, st))) break;
    if (s->nelem > 0 &&
        (e = hipMemcpyAsync(y->dslot, dslot.data(), s->nelem * 4, hipMemcpyHostToDevice, st))) break;
    if (s->nelem > 0 &&
        (e = hipMemcpyAsync(y->elem_seg, eseg.data(), s->nelem * 4, hipMemcpyHostToDevice, st))) break;
    if (lambda && (e = hipMemcpyAsync(y->lam, lambda, s->nelem * 8, hipMemcpyDeviceToDevice, st))) break;
    if ((e = hipMemcpyAsync(d_B, hB.data(), hB.size() * 8, hipMemcpyHostToDevice, st))) break;
    if ((e = hipMemcpyAsync(d_D, hD.data(), hD.size() * 8, hipMemcpyHostToDevice, st))) break;
    if ((e = hipMemsetAsync(d_bad, 0, 4, st))) break;
    if ((e = vec_fill<double>(y->diag, np, 0.0, st))) break;
    if ((e = vec_fill<double>(y->y, np, 0.0, st))) break;
    for (size_t g = 0; g < s->groups.size() && e == hipSuccess; ++g) {
      const Group& G = s->groups[g];
      const int nl = s->shape == 1   ? G.n * (G.n + 1) / 2
                     : s->shape == 2 ? G.n * (G.n + 1) * (G.n + 2) / 6
                     : s->shape == 3 ? G.n * G.n * (G.n + 1) / 2
                     : s->shape == 4 ? G.n * (G.n + 1) * (2 * G.n + 1) / 6
                                     : (int)ipow(G.n, s->dim);
      if ((e = build_l2g(G.nelem, nl, y->elem_seg + G.e0, y->d_dof_off, y->d_pdof_off, l2g + G.c0,
                         sign ? sign + G.c0 : nullptr, dirichlet, y->l2g + G.c0, d_bad, st)))
        break;
      if ((e = mark_free(G.nelem, nl, y->l2g + G.c0, y->y, st))) break;
      if (s->shape == 1)
        e = launch_diag_tri(G.P, G.nelem, s->fac64 + G.f0, y->lam ? y->lam + G.e0 : nullptr, y->lam0,
                            y->l2g + G.c0, y->diag, st);
      else if (s->shape == 2)
        e = launch_diag_tet(G.P, G.nelem, s->fac64 + G.f0, y->lam ? y->lam + G.e0 : nullptr, y->lam0,
                            y->l2g + G.c0, y->diag, st);
      else if (s->shape == 3)
        e = launch_diag_prism(G.P, G.nelem, s->fac64 + G.f0, y->lam ? y->lam + G.e0 : nullptr,
                              y->lam0, y->l2g + G.c0, y->diag, st);
      else if (s->shape == 4)
        e = launch_diag_pyr(G.P, G.nelem, s->fac64 + G.f0, y->lam ? y->lam + G.e0 : nullptr, y->lam0,
                            y->l2g + G.c0, y->diag, st);
      else
        e = launch_diag(s->dim, G.P, G.Q, G.nelem, d_B + tab_off[g], d_D + tab_off[g],
                        s->fac64 + G.f0, y->lam ? y->lam + G.e0 : nullptr, y->lam0, y->l2g + G.c0,
                        y->diag, st);
    }
    if (e) break;
    if ((e = diag_finish(y->L, y->diag, y->y, y->dinv64, y->dinv32, y->diag, st))) break;
    for (double* v : {y->b, y->x, y->r, y->p, y->y, y->u, y->s})
      if ((e = vec_fill<double>(v, np, 0.0, st))) break;
    if (e) break;
    for (float* v : {y->r32, y->p32, y->y32, y->d32, y->u32, y->s32})
      if ((e = vec_fill<float>(v, np, 0.f, st))) break;
    if (e) break;
    if ((e = vec_fill<int32_t>(y->outer_cnt, nsys, 0, st))) break;
    if ((e = vec_fill<int32_t>(y->cnt_aux, nsys, 0, st))) break;
    e = hipStreamSynchronize(st);
  } while (0);
  int bad = 0;
  if (e == hipSuccess) e = hipMemcpy(&bad, d_bad, 4, hipMemcpyDeviceToHost);
  dfree(d_bad);
  dfree(d_B);
  dfree(d_D);
  if (e != hipSuccess) return cleanup(hip_fail(e, "system setup"));
  if (bad) return cleanup(fail(NK_EINVAL, "l2g index outside its system's DOF range, or a sign other than +-1"));
  for (size_t g = 0; g < s->groups.size(); ++g) {
    y->tiles64.push_back(tune ? tune_asm_tile(y, NK_F64, (int)g, st) : 0);
    y->tiles32.push_back(tune ? tune_asm_tile(y, NK_F32, (int)g, st) : 0);
  }
  // the timing runs wrote into the work vectors: clear them again
  if ((e = vec_fill<double>(y->y, np, 0.0, st)) || (e = vec_fill<float>(y->y32, np, 0.f, st)) ||
      (e = hipStreamSynchronize(st)))
    return cleanup(hip_fail(e, "system setup"));
  *out = y;
  return NK_OK;
}

nk_status nk_system_create_batched(nk_system* out, nk_space s, int nsys, const int64_t* elem_off,
                                   const int64_t* dof_off, const int32_t* l2g,
                                   const uint8_t* dirichlet, const double* lambda, double lambda0,
                                   void* stream) {
  return system_create(out, s, nsys, elem_off, dof_off, l2g, nullptr, dirichlet, lambda, lambda0,
                       stream);
}

nk_status nk_system_create_signed(nk_system* out, nk_space s, int64_t nglobal, const int32_t* l2g,
                                  const int8_t* sign, const uint8_t* dirichlet,
                                  const double* lambda, double lambda0, void* stream) {
  if (!s) return fail(NK_EINVAL, "space is NULL");
  if (nglobal < 1) return fail(NK_EINVAL, "nglobal must be >= 1");
  const int64_t eo[2] = {0, s->nelem}, dofo[2] = {0, nglobal};
  return system_create(out, s, 1, eo, dofo, l2g, sign, dirichlet, lambda, lambda0, stream);
}

nk_status nk_system_create(nk_system* out, nk_space s, int64_t nglobal, const int32_t* l2g,
                           const uint8_t* dirichlet, const double* lambda, double lambda0,
                           void* stream) {
  if (!s) return fail(NK_EINVAL, "space is NULL");
  if (nglobal < 1) return fail(NK_EINVAL, "nglobal must be >= 1");
  const int64_t eo[2] = {0, s->nelem};
  const int64_t dofo[2] = {0, nglobal};
  return nk_system_create_batched(out, s, 1, eo, dofo, l2g, dirichlet, lambda, lambda0, stream);
}

static void union_forget(nk_system y);

nk_status nk_system_destroy(nk_system sys) {
  if (!sys) return fail(NK_EINVAL, "system is NULL");
  union_forget(sys);
  system_free(sys);
  return NK_OK;
}

// y (padded) += A x (padded) over the elements of order group g; with dots,
// each element's energy is added to its CG accumulation slot (dslot).
static hipError_t sys_op_group(nk_system y, nk_dtype t, int g, const void* x, void* out,
                               double* dots, const int32_t* seg_done, int tile, hipStream_t st) {
  nk_space s = y->space;
  if (y->sc)   // boundary system of a static condensation (hexahedral order groups)
    return sc_apply(y->sc[g], t, x, out, dots, dots ? y->dslot + s->groups[g].e0 : nullptr,
                    seg_done, st);
  const Group& G = s->groups[g];
  OpArgs a;
  a.op = OP_HELM_ASM;
  a.dim = s->dim;
  a.P = G.P;
  a.Q = G.Q;
  a.nelem = G.nelem;
  a.in = x;
  a.out = out;
  a.fac = t == NK_F64 ? (const void*)(s->fac64 + G.f0) : (const void*)(s->fac32 + G.f0);
  a.lam = y->lam ? y->lam + G.e0 : nullptr;
  a.lam0 = y->lam0;
  a.l2g = y->l2g + G.c0;
  a.dots = dots;
  a.dslot = dots ? y->dslot + G.e0 : nullptr;
  // one system: its single converged flag needs no per-element index
  a.elem_seg = seg_done && y->nsys > 1 ? y->elem_seg + G.e0 : nullptr;
  a.seg_done = seg_done;
  a.tile = tile;
  a.stream = st;
  if (s->shape == 1) return launch_tri(t, a);
  if (s->shape == 2) return launch_tet(t, a);
  if (s->shape == 3) return launch_prism(t, a);
  if (s->shape == 4) return launch_pyr(t, a);
  return launch_op(s->dim, t, a);
}

// y (padded) += A x (padded) over all elements, each order group with its
// own tuned tile.
// With several order groups the groups' launches are independent (they
// only add into out and the energy slots, atomically), so groups 1.. run on
// the system's own side streams (made at creation), forked from and joined
// back into st by events: each group alone is often too small to fill the
// GPU.  Under graph capture the fork and join become graph dependencies.
static hipError_t sys_op(nk_system y, nk_dtype t, const void* x, void* out, double* dots,
                         const int32_t* seg_done, hipStream_t st) {
  const std::vector<int>& tiles = t == NK_F64 ? y->tiles64 : y->tiles32;
  const size_t ng = y->space->groups.size();
  hipError_t e = hipSuccess;
  if (ng > 1 && y->ostreams.size() + 1 == ng) {
    if ((e = hipEventRecord(y->ofork, st))) return e;
    for (size_t g = 1; g < ng; ++g) {
      hipStream_t gs = y->ostreams[g - 1];
      if ((e = hipStreamWaitEvent(gs, y->ofork, 0)) ||
          (e = sys_op_group(y, t, (int)g, x, out, dots, seg_done, g < tiles.size() ? tiles[g] : 0, gs)) ||
          (e = hipEventRecord(y->oevents[g - 1], gs)))
        return e;
    }
    if ((e = sys_op_group(y, t, 0, x, out, dots, seg_done, tiles.empty() ? 0 : tiles[0], st))) return e;
    for (size_t g = 1; g < ng; ++g)
      if ((e = hipStreamWaitEvent(st, y->oevents[g - 1], 0))) return e;
    return hipSuccess;
  }
  for (size_t g = 0; g < ng; ++g) {
    e = sys_op_group(y, t, (int)g, x, out, dots, seg_done, g < tiles.size() ? tiles[g] : 0, st);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

nk_status nk_system_apply(nk_system sys, nk_dtype t, const void* x, void* yv, void* stream) {
  if (!sys) return fail(NK_EINVAL, "system is NULL");
  if (t != NK_F64 && t != NK_F32) return fail(NK_EINVAL, "bad dtype");
  NK_CHECK(check_buf(x, sys->nuser * dsize(t), "x"));
  NK_CHECK(check_buf(yv, sys->nuser * dsize(t), "y"));
  hipStream_t st = (hipStream_t)stream;
  const int64_t np = sys->L.npad;
  hipError_t e;
  if (t == NK_F64) {
    if ((e = pad_in<double>(sys->nsys, sys->d_dof_off, sys->d_pdof_off, sys->L, (const double*)x,
                            sys->dinv64, sys->p, st)) ||
        (e = vec_fill<double>(sys->y, np, 0.0, st)) ||
        (e = sys_op(sys, t, sys->p, sys->y, nullptr, nullptr, st)) ||
        (e = pad_out<double>(sys->nsys, sys->d_dof_off, sys->d_pdof_off, sys->nuser, sys->y,
                             (double*)yv, st)))
      return hip_fail(e, "system apply");
  } else {
    if ((e = pad_in<float>(sys->nsys, sys->d_dof_off, sys->d_pdof_off, sys->L, (const float*)x,
                           sys->dinv64, sys->p32, st)) ||
        (e = vec_fill<float>(sys->y32, np, 0.f, st)) ||
        (e = sys_op(sys, t, sys->p32, sys->y32, nullptr, nullptr, st)) ||
        (e = pad_out<float>(sys->nsys, sys->d_dof_off, sys->d_pdof_off, sys->nuser, sys->y32,
                            (float*)yv, st)))
      return hip_fail(e, "system apply");
  }
  // the padded work vectors are shared with solves on the system's own stream
  if ((e = hipStreamSynchronize(st))) return hip_fail(e, "system apply");
  return NK_OK;
}

// ------------------------------------------------ allocation-free apply
// Staging of nk_system_apply_noalloc: the padded input and output vectors of
// the assembled operator live in this file-scope device array instead of the
// system's work vectors.  Each GPU the library runs on holds its own copy
// (kScratchBytes) until the process ends.  Host code never passes `scratch`
// itself to a kernel: its device address is looked up once per device
// (scratch_base) and only that address is used.
constexpr size_t kScratchBytes = size_t(64) << 20;
constexpr int kScratchMaxDevices = 64;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];
static std::mutex g_scratch_mu;
static void* g_scratch_dev[kScratchMaxDevices] = {};

// Device address of `scratch` on the current device `dev`, looked up on the
// first call on that device (with it current) and kept.
static nk_status scratch_base(int dev, void** out) {
  if (dev < 0 || dev >= kScratchMaxDevices) return fail(NK_EDEVICE, "device index out of range");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_dev[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
    if (!p) return fail(NK_EHIP, "hipGetSymbolAddress(scratch) returned NULL");
    g_scratch_dev[dev] = p;
  }
  *out = g_scratch_dev[dev];
  return NK_OK;
}

nk_status nk_system_apply_noalloc(nk_system sys, nk_dtype t, const void* x, void* yv,
                                  void* stream) {
  if (!sys) return fail(NK_EINVAL, "system is NULL");
  if (t != NK_F64 && t != NK_F32) return fail(NK_EINVAL, "bad dtype");
  NK_CHECK(check_buf(x, sys->nuser * dsize(t), "x"));
  NK_CHECK(check_buf(yv, sys->nuser * dsize(t), "y"));
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  if (dev != sys->device)
    return fail(NK_EINVAL, "the system's device must be current (system on device " +
                               std::to_string(sys->device) + ", current " + std::to_string(dev) + ")");
  const int64_t np = sys->L.npad;
  const size_t need = 2 * (size_t)np * dsize(t);
  if (need > kScratchBytes)
    return fail(NK_EINVAL, "system too large for the static scratch: needs " + std::to_string(need) +
                               " bytes (two padded vectors of " + std::to_string(np) +
                               " entries), the maximum is " + std::to_string(kScratchBytes) +
                               " bytes");
  void* base = nullptr;
  NK_CHECK(scratch_base(dev, &base));
  hipStream_t st = (hipStream_t)stream;
  if (t == NK_F64) {
    double* xin = (double*)base;
    double* yout = xin + np;
    if ((e = pad_in<double>(sys->nsys, sys->d_dof_off, sys->d_pdof_off, sys->L, (const double*)x,
                            sys->dinv64, xin, st)) ||
        (e = vec_fill<double>(yout, np, 0.0, st)) ||
        (e = sys_op(sys, t, xin, yout, nullptr, nullptr, st)) ||
        (e = pad_out<double>(sys->nsys, sys->d_dof_off, sys->d_pdof_off, sys->nuser, yout,
                             (double*)yv, st)))
      return hip_fail(e, "system apply (no allocation)");
  } else {
    float* xin = (float*)base;
    float* yout = xin + np;
    if ((e = pad_in<float>(sys->nsys, sys->d_dof_off, sys->d_pdof_off, sys->L, (const float*)x,
                           sys->dinv64, xin, st)) ||
        (e = vec_fill<float>(yout, np, 0.f, st)) ||
        (e = sys_op(sys, t, xin, yout, nullptr, nullptr, st)) ||
        (e = pad_out<float>(sys->nsys, sys->d_dof_off, sys->d_pdof_off, sys->nuser, yout,
                            (float*)yv, st)))
      return hip_fail(e, "system apply (no allocation)");
  }
  return NK_OK;
}

nk_status nk_assemble(nk_system sys, const double* y_loc, double* b, void* stream) {
  if (!sys) return fail(NK_EINVAL, "system is NULL");
  nk_space s = sys->space;
  NK_CHECK(check_buf(y_loc, (size_t)s->ncoeff * 8, "y_loc"));
  NK_CHECK(check_buf(b, sys->nuser * 8, "b"));
  hipStream_t st = (hipStream_t)stream;
  hipError_t e;
  if ((e = vec_fill<double>(sys->y, sys->L.npad, 0.0, st)) ||
      (e = scatter_add(s->ncoeff, 1, sys->l2g, y_loc, sys->y, st)) ||
      (e = pad_out<double>(sys->nsys, sys->d_dof_off, sys->d_pdof_off, sys->nuser, sys->y, b, st)) ||
      (e = hipStreamSynchronize(st)))
    return hip_fail(e, "assemble");
  return NK_OK;
}

nk_status nk_gather(nk_system sys, const double* x, double* x_loc, void* stream) {
  if (!sys) return fail(NK_EINVAL, "system is NULL");
  nk_space s = sys->space;
  NK_CHECK(check_buf(x, sys->nuser * 8, "x"));
  NK_CHECK(check_buf(x_loc, (size_t)s->ncoeff * 8, "x_loc"));
  hipStream_t st = (hipStream_t)stream;
  hipError_t e;
  // Dirichlet entries are gathered as they are (not masked): the reported
  // diagonal is nonzero on every row of a definite system, so it serves as an
  // all-pass mask.
  if ((e = pad_in<double>(sys->nsys, sys->d_dof_off, sys->d_pdof_off, sys->L, x, sys->diag,
                          sys->p, st)) ||
      (e = gather_user(s->ncoeff, 1, sys->l2g, sys->p, x_loc, st)) ||
      (e = hipStreamSynchronize(st)))
    return hip_fail(e, "gather");
  return NK_OK;
}

nk_status nk_system_diagonal(nk_system sys, double* diag, void* stream) {
  if (!sys) return fail(NK_EINVAL, "system is NULL");
  NK_CHECK(check_buf(diag, sys->nuser * 8, "diag"));
  hipStream_t st = (hipStream_t)stream;
  hipError_t e;
  if ((e = pad_out<double>(sys->nsys, sys->d_dof_off, sys->d_pdof_off, sys->nuser, sys->diag, diag,
                           st)) ||
      (e = hipStreamSynchronize(st)))
    return hip_fail(e, "diagonal");
  return NK_OK;
}

// ------------------------------------------------------------------ solve
// CG iterations per captured graph: a multiple of 6, the period of the
// rotating reduction sets (cg.hip), so every launch starts on set 0.
static int graph_iters() {
  const char* v = std::getenv("NK_GRAPH_ITERS");
  const int k = v ? std::atoi(v) : 18;
  return std::min(std::max((k + 5) / 6 * 6, 6), 252);
}

static double inner_tol() {
  const char* v = std::getenv("NK_INNER_TOL");
  const double t = v ? std::atof(v) : 1e-4;
  return (t > 0.0 && t < 1.0) ? t : 1e-4;
}

// Delta slot set q of precision T's state.
static double* dset(nk_system y, const CgState& st, int q) {
  return st.dsl + (int64_t)q * y->nsys * kSlots;
}

// CG iteration j (of a graph launch) in precision T on the system's stream:
// the update (which forms its step from the slot sums) and the assembled
// operator w = A u, whose element energies go to delta set j+1.
template <typename T>
static hipError_t cg_iteration(nk_system y, int j) {
  const bool f64 = std::is_same<T, double>::value;
  CgState& st = f64 ? y->st64 : y->st32;
  T* x = f64 ? (T*)y->x : (T*)y->d32;
  T* r = f64 ? (T*)y->r : (T*)y->r32;
  T* u = f64 ? (T*)y->u : (T*)y->u32;
  T* p = f64 ? (T*)y->p : (T*)y->p32;
  T* s = f64 ? (T*)y->s : (T*)y->s32;
  T* w = f64 ? (T*)y->y : (T*)y->y32;
  const T* dinv = f64 ? (const T*)y->dinv64 : (const T*)y->dinv32;
  hipError_t e;
  if ((e = cg_update<T>(y->L, st, y->nsys, j, f64, nullptr, x, r, u, p, s, w, dinv, y->cs)))
    return e;
  return sys_op(y, f64 ? NK_F64 : NK_F32, u, w, dset(y, st, (j + 1) & 1), st.done, y->cs);
}

// First step of a CG solve in precision T: r = b - w (w = A x0 or 0),
// u = M^{-1} r, w = A u, and the scalars the first update reads.  Systems
// whose skip flag is set (or whose residual already meets tol2) stop at once.
template <typename T>
static hipError_t cg_begin(nk_system y, const double* b, double tau2, const int32_t* skip) {
  const bool f64 = std::is_same<T, double>::value;
  CgState& st = f64 ? y->st64 : y->st32;
  T* r = f64 ? (T*)y->r : (T*)y->r32;
  T* u = f64 ? (T*)y->u : (T*)y->u32;
  T* p = f64 ? (T*)y->p : (T*)y->p32;
  T* s = f64 ? (T*)y->s : (T*)y->s32;
  T* w = f64 ? (T*)y->y : (T*)y->y32;
  const T* dinv = f64 ? (const T*)y->dinv64 : (const T*)y->dinv32;
  const int ns = y->nsys;
  hipError_t e;
  if ((e = vec_fill<double>(st.gsl, (int64_t)3 * ns * 2 * kSlots, 0.0, y->cs)) ||
      (e = vec_fill<double>(st.dsl, (int64_t)2 * ns * kSlots, 0.0, y->cs)))
    return e;
  if ((e = cg_start<T>(y->L, st, ns, b, w, r, u, p, s, dinv, y->cs))) return e;
  if ((e = sys_op(y, f64 ? NK_F64 : NK_F32, u, w, dset(y, st, 0), nullptr, y->cs))) return e;
  return cg_begin_scalars(st, ns, tau2, skip, y->outer_tol2, y->outer_rr, y->cs);
}

template <typename T>
static hipError_t ensure_graph(nk_system y) {
  const bool f64 = std::is_same<T, double>::value;
  hipGraphExec_t& ge = f64 ? y->g64 : y->g32;
  int& gi = f64 ? y->g64_iters : y->g32_iters;
  const int k = graph_iters();
  if (ge && gi == k) return hipSuccess;
  if (ge) {
    (void)hipGraphExecDestroy(ge);
    ge = nullptr;
  }
  hipGraph_t g = nullptr;
  hipError_t e = hipStreamBeginCapture(y->cs, hipStreamCaptureModeThreadLocal);
  if (e) return e;
  hipError_t e2 = hipSuccess;
  for (int i = 0; i < k && e2 == hipSuccess; ++i) e2 = cg_iteration<T>(y, i);
  e = hipStreamEndCapture(y->cs, &g);
  if (e2) {
    if (g) (void)hipGraphDestroy(g);
    return e2;
  }
  if (e) return e;
  e = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (e) return e;
  gi = k;
  return hipSuccess;
}

// Copy per-system iteration budgets to the device state of precision T.
static hipError_t set_budgets(nk_system y, const CgState& st, const std::vector<int>& budget) {
  for (int i = 0; i < y->nsys; ++i) y->h_budget[i] = budget[i];
  return hipMemcpyAsync(st.maxit, y->h_budget, y->nsys * 4, hipMemcpyHostToDevice, y->cs);
}

// Run graph launches of CG iterations until every system reports done; the
// largest budget bounds the number of launches.
template <typename T>
static hipError_t cg_loop(nk_system y, int max_budget, const int32_t* done_dev) {
  hipError_t e = ensure_graph<T>(y);
  if (e) return e;
  const hipGraphExec_t ge = std::is_same<T, double>::value ? y->g64 : y->g32;
  const int k = std::is_same<T, double>::value ? y->g64_iters : y->g32_iters;
  const int64_t max_launch = (int64_t)max_budget / k + 2;
  for (int64_t l = 0; l < max_launch; ++l) {
    if ((e = hipGraphLaunch(ge, y->cs))) return e;
    if ((e = hipMemcpyAsync(y->h_flags, done_dev, y->nsys * 4, hipMemcpyDeviceToHost, y->cs)))
      return e;
    if ((e = hipStreamSynchronize(y->cs))) return e;
    bool all = true;
    for (int i = 0; i < y->nsys; ++i) all = all && y->h_flags[i] != 0;
    if (all) break;
  }
  return hipSuccess;
}

// True FP64 residual of the current x: rr_true = ||b - A x||^2 per system
// (r holds b - A x on free DOFs, y is left zero).
static hipError_t true_residual(nk_system y) {
  CgState chk;
  chk.rr = y->rr_true;
  chk.tol2 = y->outer_tol2;
  chk.cnt = y->cnt_aux;
  hipError_t e;
  if ((e = vec_fill<double>(y->y, y->L.npad, 0.0, y->cs))) return e;
  if ((e = sys_op(y, NK_F64, y->x, y->y, nullptr, nullptr, y->cs))) return e;
  return cg_residual(y->L, chk, y->b, y->y, y->dinv64, y->r, nullptr, y->part, y->cs);
}

// Relative residual as reported in nk_solve_info; convergence decisions on
// the host use this same expression, so NK_OK implies rel_resid <= rtol.
static double rel_of(double rr, double bb) { return bb > 0.0 ? std::sqrt(rr / bb) : std::sqrt(rr); }

// Read an nsys-long device array through the pinned staging buffer.
template <typename V>
static hipError_t read_sys(nk_system y, const V* dev, std::vector<V>& out) {
  out.resize(y->nsys);
  V* h = sizeof(V) == 8 ? (V*)y->h_d : (V*)y->h_flags;
  hipError_t e;
  if ((e = hipMemcpyAsync(h, dev, y->nsys * sizeof(V), hipMemcpyDeviceToHost, y->cs))) return e;
  if ((e = hipStreamSynchronize(y->cs))) return e;
  for (int i = 0; i < y->nsys; ++i) out[i] = h[i];
  return hipSuccess;
}

// Read an int32 and an FP64 nsys-long device array (or, with dd null, two
// int32 arrays) through the pinned staging buffers with one synchronisation:
// the solve loops check flags and residuals after every graph launch, and
// each synchronisation leaves the GPU idle while the host looks.
static hipError_t read_sys2(nk_system y, const int32_t* di, std::vector<int32_t>& oi,
                            const double* dd, std::vector<double>& od,
                            const int32_t* di2 = nullptr, std::vector<int32_t>* oi2 = nullptr) {
  const int ns = y->nsys;
  hipError_t e;
  if ((e = hipMemcpyAsync(y->h_flags, di, ns * 4, hipMemcpyDeviceToHost, y->cs))) return e;
  if (dd && (e = hipMemcpyAsync(y->h_d, dd, ns * 8, hipMemcpyDeviceToHost, y->cs))) return e;
  if (di2 && (e = hipMemcpyAsync(y->h_flags + ns, di2, ns * 4, hipMemcpyDeviceToHost, y->cs))) return e;
  if ((e = hipStreamSynchronize(y->cs))) return e;
  oi.assign(y->h_flags, y->h_flags + ns);
  if (dd) od.assign(y->h_d, y->h_d + ns);
  if (di2) oi2->assign(y->h_flags + ns, y->h_flags + 2 * ns);
  return hipSuccess;
}

// FP64 CG restarted from the current x while the true residual of a system
// is above rtol and its budget lasts: the recursive residual the iteration
// stops on drifts from b - A x by rounding, so one restart (a few
// iterations) usually closes the gap.  On return rr_true holds each system's
// true squared residual and stat its status.
static hipError_t solve_f64(nk_system y, double rtol, int maxit, std::vector<int>& iters,
                            std::vector<int32_t>& stat, std::vector<double>& rr) {
  const int ns = y->nsys;
  const int kMaxPasses = 8;
  std::vector<double> bb;
  std::vector<int32_t> it_dev, st_dev;
  std::vector<int> budget(ns, maxit);
  std::vector<char> fin(ns, 0);
  hipError_t e;
  if ((e = vec_norm2(y->L, y->b, y->part, y->cnt_aux, y->bb, rtol, y->st64.tol2, y->cs))) return e;
  if ((e = vec_fill<int32_t>(y->outer_done, ns, 0, y->cs))) return e;
  if ((e = read_sys(y, y->bb, bb))) return e;
  stat.assign(ns, NK_OK);
  for (int pass = 0; pass < kMaxPasses; ++pass) {
    int maxb = 0;
    for (int i = 0; i < ns; ++i) {
      budget[i] = fin[i] ? 0 : maxit - iters[i];
      maxb = std::max(maxb, budget[i]);
    }
    if ((e = set_budgets(y, y->st64, budget))) return e;
    if ((e = vec_fill<double>(y->y, y->L.npad, 0.0, y->cs))) return e;
    if ((e = sys_op(y, NK_F64, y->x, y->y, nullptr, nullptr, y->cs))) return e;
    if ((e = cg_begin<double>(y, y->b, 0.0, y->outer_done))) return e;
    if ((e = cg_loop<double>(y, maxb, y->st64.done))) return e;
    std::vector<double> unused;
    if ((e = read_sys2(y, y->st64.iters, it_dev, nullptr, unused, y->st64.status, &st_dev))) return e;
    if ((e = true_residual(y)) || (e = read_sys(y, y->rr_true, rr))) return e;
    bool again = false;
    for (int i = 0; i < ns; ++i) {
      if (fin[i]) continue;
      iters[i] += it_dev[i];
      const bool met = rel_of(rr[i], bb[i]) <= rtol;
      if (st_dev[i] != NK_OK || met || iters[i] >= maxit) {
        fin[i] = 1;
        stat[i] = st_dev[i] != NK_OK ? st_dev[i] : met ? NK_OK : NK_ENOCONV;
      } else {
        again = true;
      }
    }
    if (!again) break;
    for (int i = 0; i < ns; ++i) y->h_budget[i] = fin[i];
    if ((e = hipMemcpyAsync(y->outer_done, y->h_budget, ns * 4, hipMemcpyHostToDevice, y->cs)) ||
        (e = hipStreamSynchronize(y->cs)))
      return e;
  }
  for (int i = 0; i < ns; ++i)
    if (!fin[i]) stat[i] = NK_ENOCONV;
  return hipSuccess;
}

// FP64 iterative refinement around an FP32 inner CG.  maxit bounds the
// inner iterations summed over refinement steps; a system whose budget runs
// out gets an infinite outer tolerance (so it is skipped from then on) and
// status NK_ENOCONV.  The outer residual that ends the loop is the true FP64
// residual of the returned x (x does not change after it), left in rr_true.
static hipError_t solve_refined(nk_system y, double rtol, int maxit, std::vector<int>& iters,
                                std::vector<int>& outer, std::vector<int32_t>& stat,
                                std::vector<double>& rr) {
  const int ns = y->nsys;
  const int64_t np = y->L.npad;
  hipStream_t cs = y->cs;
  CgState outer_st;
  outer_st.rr = y->outer_rr;
  outer_st.tol2 = y->outer_tol2;
  outer_st.done = y->outer_done;
  outer_st.status = y->outer_status;
  outer_st.cnt = y->outer_cnt;
  std::vector<double> bb;
  std::vector<int32_t> done, it_dev;
  std::vector<int> budget(ns, 0);
  std::vector<char> spent(ns, 0);
  hipError_t e;
  // the device stops on rr <= (rtol (1 - 1e-14))^2 ||b||^2, a hair inside
  // the host's rel_of(rr, bb) <= rtol, so the two never disagree by rounding
  const double rtol_dev = rtol * (1.0 - 1e-14);
  if ((e = vec_norm2(y->L, y->b, y->part, y->cnt_aux, y->bb, rtol_dev, y->outer_tol2, cs)))
    return e;
  if ((e = read_sys(y, y->bb, bb))) return e;
  const double tau = inner_tol();
  const int max_outer = 60;
  bool all = false;
  for (int k = 0; k <= max_outer; ++k) {
    if ((e = vec_fill<double>(y->y, np, 0.0, cs))) return e;
    if ((e = sys_op(y, NK_F64, y->x, y->y, nullptr, nullptr, cs))) return e;
    if ((e = cg_residual(y->L, outer_st, y->b, y->y, y->dinv64, y->r, nullptr, y->part, cs)))
      return e;
    if ((e = read_sys(y, y->outer_done, done))) return e;
    all = true;
    int maxb = 0;
    for (int i = 0; i < ns; ++i) {
      all = all && done[i] != 0;
      budget[i] = done[i] ? 0 : maxit - iters[i];
      maxb = std::max(maxb, budget[i]);
    }
    if (all || k == max_outer) break;
    for (int i = 0; i < ns; ++i)
      if (!done[i]) outer[i] += 1;
    if ((e = set_budgets(y, y->st32, budget))) return e;
    if ((e = vec_fill<float>(y->d32, np, 0.f, cs))) return e;
    if ((e = vec_fill<float>(y->y32, np, 0.f, cs))) return e;
    if ((e = cg_begin<float>(y, y->r, tau * tau, y->outer_done))) return e;
    if ((e = cg_loop<float>(y, maxb, y->st32.done))) return e;
    if ((e = read_sys(y, y->st32.iters, it_dev))) return e;
    bool newly_spent = false;
    for (int i = 0; i < ns; ++i) {
      if (done[i]) continue;
      iters[i] += it_dev[i];
      if (iters[i] >= maxit && !spent[i]) spent[i] = newly_spent = true;
    }
    if ((e = cg_correct(y->L, y->outer_done, y->d32, y->x, cs))) return e;
    if (newly_spent) {
      // out of budget: this system's x is final after the correction above
      for (int i = 0; i < ns; ++i) y->h_d[i] = spent[i] ? HUGE_VAL : rtol_dev * rtol_dev * bb[i];
      if ((e = hipMemcpyAsync(y->outer_tol2, y->h_d, ns * 8, hipMemcpyHostToDevice, cs))) return e;
      if ((e = hipStreamSynchronize(cs))) return e;
    }
  }
  if ((e = read_sys(y, y->outer_rr, rr))) return e;
  stat.assign(ns, NK_OK);
  for (int i = 0; i < ns; ++i) stat[i] = rel_of(rr[i], bb[i]) <= rtol ? NK_OK : NK_ENOCONV;
  return hipSuccess;
}

// Residual reduction between reliable updates.  Measured on 24^3 curved
// hexes (FP32 iterations / solve time): 0.3 takes 16-17 updates and the
// fewest FP32 iterations (P=8: 1536, P=6: 999); 0.1 takes 9 (1616, 1004);
// 0.03 lets the FP32 recurrence drift so far that P=8 needs 3367.
static double reliable_delta() {
  const char* v = std::getenv("NK_RELIABLE_DELTA");
  const double d = v ? std::atof(v) : 0.3;
  return (d > 0.0 && d < 1.0) ? d : 0.3;
}

static bool refine_by_restart() {
  const char* v = std::getenv("NK_REFINE");
  return v && std::strcmp(v, "restart") == 0;
}

// FP32 CG with reliable updates inside FP64: one FP32 Jacobi-PCG whose
// recursive residual is replaced by the true FP64 residual b - A x whenever
// every active system's FP32 residual has fallen by reliable_delta() since
// the last replacement, or a system's FP32 iteration stopped; the FP32
// solution increment is then added to the FP64 x and cleared.  The search
// directions are kept across the replacement (the last step's alpha and beta
// are recomputed from the new residual), so no Krylov information is lost as
// it is when the inner solve restarts.  The loop ends on the true FP64
// residual of the returned x (left in rr); maxit bounds the FP32 iterations.
static hipError_t solve_reliable(nk_system y, double rtol, int maxit, std::vector<int>& iters,
                                 std::vector<int>& outer, std::vector<int32_t>& stat,
                                 std::vector<double>& rr) {
  const int ns = y->nsys;
  const int64_t np = y->L.npad;
  hipStream_t cs = y->cs;
  CgState outer_st;
  outer_st.rr = y->outer_rr;
  outer_st.tol2 = y->outer_tol2;
  outer_st.done = y->outer_done;
  outer_st.status = y->outer_status;
  outer_st.cnt = y->outer_cnt;
  const double rtol_dev = rtol * (1.0 - 1e-14);
  const double d2 = reliable_delta() * reliable_delta();
  std::vector<double> bb, rr_last, rr32;
  std::vector<int32_t> done, done32, it_dev, st_dev;
  std::vector<char> fin(ns, 0);
  stat.assign(ns, NK_OK);
  hipError_t e;
  auto true_resid = [&]() -> hipError_t {
    hipError_t e2;
    if ((e2 = vec_fill<double>(y->y, np, 0.0, cs))) return e2;
    if ((e2 = sys_op(y, NK_F64, y->x, y->y, nullptr, nullptr, cs))) return e2;
    if ((e2 = cg_residual(y->L, outer_st, y->b, y->y, y->dinv64, y->r, nullptr, y->part, cs)))
      return e2;
    return read_sys2(y, y->outer_done, done, y->outer_rr, rr_last);
  };
  if ((e = vec_norm2(y->L, y->b, y->part, y->cnt_aux, y->bb, rtol_dev, y->outer_tol2, cs))) return e;
  if ((e = read_sys(y, y->bb, bb))) return e;
  if ((e = true_resid())) return e;
  bool all = true;
  for (int i = 0; i < ns; ++i) all = all && done[i] != 0;
  const bool began = !all;
  if (began) {
    if ((e = set_budgets(y, y->st32, std::vector<int>(ns, maxit)))) return e;
    if ((e = vec_fill<float>(y->d32, np, 0.f, cs))) return e;
    if ((e = vec_fill<float>(y->y32, np, 0.f, cs))) return e;
    // the FP32 iteration stops at half the target residual (tol2 = outer_tol2 / 4)
    if ((e = cg_begin<float>(y, y->r, 1e-300, y->outer_done))) return e;
    if ((e = ensure_graph<float>(y))) return e;
    for (int i = 0; i < ns; ++i)
      if (!done[i]) outer[i] = 1;
    const int64_t max_launch = (int64_t)maxit / y->g32_iters + 2;
    int64_t launches = 0;
    for (int upd = 0; upd < 10000; ++upd) {
      // FP32 iterations until a reliable update is due
      bool due = false;
      while (!due) {
        if (launches++ >= max_launch) {
          due = true;
          break;
        }
        if ((e = hipGraphLaunch(y->g32, cs))) return e;
        if ((e = read_sys2(y, y->st32.done, done32, y->st32.rr, rr32))) return e;
        bool progressed = true, any_stopped = false, active = false;
        for (int i = 0; i < ns; ++i) {
          if (done[i] || fin[i]) continue;
          active = true;
          any_stopped = any_stopped || done32[i] != 0;
          progressed = progressed && rr32[i] <= d2 * rr_last[i];
        }
        due = !active || any_stopped || progressed;
      }
      // fold the FP32 increment into x and take the true residual
      if ((e = cg_correct(y->L, y->outer_done, y->d32, y->x, cs))) return e;
      if ((e = vec_fill<float>(y->d32, np, 0.f, cs))) return e;
      if ((e = true_resid())) return e;
      std::vector<double> unused;
      if ((e = read_sys2(y, y->st32.iters, it_dev, nullptr, unused, y->st32.status, &st_dev))) return e;
      bool newly_fin = false;
      all = true;
      for (int i = 0; i < ns; ++i) {
        if (done[i] || fin[i]) continue;
        if (it_dev[i] >= maxit || st_dev[i] != NK_OK || launches > max_launch) {
          fin[i] = newly_fin = true;   // budget spent or breakdown: x is final
          stat[i] = st_dev[i] != NK_OK ? st_dev[i] : NK_ENOCONV;
          continue;
        }
        all = false;
        outer[i] += 1;
      }
      if (newly_fin) {
        // finished systems get an infinite tolerance: skipped from now on
        for (int i = 0; i < ns; ++i) y->h_d[i] = fin[i] ? HUGE_VAL : rtol_dev * rtol_dev * bb[i];
        if ((e = hipMemcpyAsync(y->outer_tol2, y->h_d, ns * 8, hipMemcpyHostToDevice, cs)) ||
            (e = hipStreamSynchronize(cs)))
          return e;
      }
      if (all) break;
      // the FP32 residual becomes the true one; p and s are kept, and the
      // next update redoes the last step from the new gamma and delta
      CgState& s32 = y->st32;
      if ((e = vec_fill<double>(s32.gsl, (int64_t)ns * 2 * kSlots, 0.0, cs)) ||
          (e = vec_fill<double>(s32.dsl, (int64_t)ns * kSlots, 0.0, cs)))
        return e;
      if ((e = cg_reliable(y->L, s32, ns, y->r, y->r32, y->u32, y->y32, y->dinv32, cs))) return e;
      if ((e = sys_op(y, NK_F32, y->u32, y->y32, dset(y, s32, 0), y->outer_done, cs))) return e;
      if ((e = cg_rearm(s32, ns, y->outer_done, cs))) return e;
    }
  }
  it_dev.assign(ns, 0);
  if (began && (e = read_sys(y, y->st32.iters, it_dev))) return e;
  rr = rr_last;
  for (int i = 0; i < ns; ++i) {
    iters[i] = it_dev[i];
    if (stat[i] == NK_OK && !(rel_of(rr[i], bb[i]) <= rtol)) stat[i] = NK_ENOCONV;
  }
  return hipSuccess;
}

// Per-system results of one solve of a (possibly batched) system.
struct SolveOut {
  std::vector<int> iters, outer;
  std::vector<int32_t> stat;
  std::vector<double> rr, bb;
};

// Solve on the padded work vectors y->b (right-hand side) and y->x (initial
// guess, then solution), already filled, on the system's private stream.
static hipError_t solve_padded(nk_system y, nk_solve_mode mode, double rtol, int maxit,
                               SolveOut& o) {
  o.iters.assign(y->nsys, 0);
  o.outer.assign(y->nsys, 0);
  hipError_t e = mode == NK_SOLVE_F64 ? solve_f64(y, rtol, maxit, o.iters, o.stat, o.rr)
                 : refine_by_restart()
                     ? solve_refined(y, rtol, maxit, o.iters, o.outer, o.stat, o.rr)
                     : solve_reliable(y, rtol, maxit, o.iters, o.outer, o.stat, o.rr);
  if (e) return e;
  return read_sys(y, y->bb, o.bb);
}

static nk_status check_solve_args(nk_solve_mode mode, double rtol, int maxit) {
  if (mode != NK_SOLVE_F64 && mode != NK_SOLVE_F32_REFINED && mode != NK_SOLVE_CONDENSED &&
      mode != NK_SOLVE_CONDENSED_F32_REFINED)
    return fail(NK_EINVAL, "bad mode");
  if (!(rtol > 0.0) || rtol >= 1.0) return fail(NK_EINVAL, "rtol must be in (0, 1)");
  if (maxit < 1) return fail(NK_EINVAL, "maxit must be >= 1");
  return NK_OK;
}

static void fill_info(nk_solve_info* info, const SolveOut& o, int i, nk_solve_mode mode, double ms) {
  info->iters = o.iters[i];
  info->outer_iters = mode == NK_SOLVE_F32_REFINED ? o.outer[i] : 0;
  info->rel_resid = rel_of(o.rr[i], o.bb[i]);
  info->solve_ms = ms;
  info->status = o.stat[i];
}

// ---------------------------------------------------- static condensation
// Section 2.1: the assembled hexahedral system condensed onto the elemental
// boundary DOFs.  The boundary system is an ordinary assembled system over
// the boundary DOFs plus one dummy Dirichlet DOF that every interior mode
// maps to (so the assembled kernels gather 0 there and scatter nothing); its
// operator is the fused condensed one of condense.hip, its Jacobi
// preconditioner the diagonal of S.

static void cond_free(CondData*& c) {
  if (!c) return;
  if (c->bsys) system_free(c->bsys);
  dfree(c->bmap);
  dfree(c->iidx);
  dfree(c->ainv);
  dfree(c->ainv32);
  dfree(c->t);
  dfree(c->zero);
  delete c;
  c = nullptr;
}

static nk_status cond_check(nk_system y) {
  nk_space s = y->space;
  if (y->nsys != 1) return fail(NK_EUNSUPPORTED, "static condensation takes a one-system (not batched) system");
  if (s->shape != 0 || s->dim != 3)
    return fail(NK_EUNSUPPORTED, "static condensation is built for hexahedral spaces");
  for (const Group& G : s->groups)
    if (G.P < kCondMinP || G.P > kCondMaxP || G.Q != G.P + 2)
      return fail(NK_EUNSUPPORTED, "static condensation is built for 2 <= P <= 6 with Q = P + 2");
  return NK_OK;
}

// Time the two fused-kernel variants of one precision on the boundary
// system (five launches each, after a warm-up) and keep the faster.  The
// timing runs write into the boundary system's work vectors, cleared after.
static hipError_t cond_pick_variant(CondData* c, int g, nk_dtype t, hipStream_t st) {
  nk_system z = c->bsys;
  CondOp& op = c->ops[g];
  const int64_t np = z->L.npad;
  void* in = t == NK_F64 ? (void*)c->zero : (void*)z->s32;
  void* out = t == NK_F64 ? (void*)z->y : (void*)z->y32;
  int& var = t == NK_F64 ? op.variant : op.variant32;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t e;
  if (t == NK_F32 && (e = vec_fill<float>(z->s32, np, 0.f, st))) return e;
  if ((e = hipEventCreate(&e0))) return e;
  if ((e = hipEventCreate(&e1))) {
    (void)hipEventDestroy(e0);
    return e;
  }
  float best = 0.f;
  int pick = 0;
  for (int v = 0; v < 2 && e == hipSuccess; ++v) {
    var = v;
    e = sc_apply(op, t, in, out, nullptr, nullptr, nullptr, st);   // warm-up
    if (e == hipSuccess) e = hipEventRecord(e0, st);
    for (int r = 0; r < 5 && e == hipSuccess; ++r)
      e = sc_apply(op, t, in, out, nullptr, nullptr, nullptr, st);
    if (e == hipSuccess) e = hipEventRecord(e1, st);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float ms = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    if (e == hipSuccess && (v == 0 || ms < best)) {
      best = ms;
      pick = v;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  var = pick;
  if (e == hipSuccess)
    e = t == NK_F64 ? vec_fill<double>(z->y, np, 0.0, st) : vec_fill<float>(z->y32, np, 0.f, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  return e;
}

// The FP32 copy of the inverses and the FP32 kernel choice (first refined
// condensed solve of a system).
static nk_status cond_build_f32(CondData* c, hipStream_t st) {
  if (c->ainv32) return NK_OK;
  int64_t n = 0;
  for (const CondOp& op : c->ops) {
    const int ni = (op.P - 1) * (op.P - 1) * (op.P - 1);
    n += op.nelem * sc_packed(ni);
  }
  n = std::max<int64_t>(n, 1);
  hipError_t e;
  if ((e = dmalloc(&c->ainv32, n))) return hip_fail(e, "hipMalloc");
  if ((e = cast_copy(c->ainv, c->ainv32, n, st)) || (e = hipStreamSynchronize(st))) {
    dfree(c->ainv32);
    return hip_fail(e, "condensation setup");
  }
  for (CondOp& op : c->ops) op.ainv32 = c->ainv32 + (op.ainv - c->ainv);
  for (size_t g = 0; g < c->ops.size(); ++g)
    if ((e = cond_pick_variant(c, (int)g, NK_F32, st))) return hip_fail(e, "condensation setup");
  return NK_OK;
}

// Build the boundary system and the interior inverses of y (once).  Each
// order group of the space has its own interior modes, inverses and fused
// kernel; the boundary numbering is global.
static nk_status cond_build(nk_system y, hipStream_t st) {
  if (y->cond) return NK_OK;
  NK_CHECK(cond_check(y));
  nk_space s = y->space;
  const int ng = (int)s->groups.size();
  const int64_t E = s->nelem, nloc = s->ncoeff, nu = y->nuser;
  hipError_t e;
  // the internal map of a one-system system numbers DOFs as the caller does
  std::vector<int32_t> m(nloc);
  if ((e = hipMemcpyAsync(m.data(), y->l2g, nloc * 4, hipMemcpyDeviceToHost, st)) ||
      (e = hipStreamSynchronize(st)))
    return hip_fail(e, "condensation setup");
  std::vector<std::vector<uint8_t>> inner(ng);
  std::vector<int64_t> ioff(ng + 1, 0), aoff(ng + 1, 0);
  int64_t max_loc = 1, max_full = 1;
  for (int g = 0; g < ng; ++g) {
    const Group& G = s->groups[g];
    const int P = G.P, n = P + 1, ni = (P - 1) * (P - 1) * (P - 1);
    inner[g].assign(n * n * n, 0);
    for (int r = 0; r < n; ++r)
      for (int hi = 0; hi < n; ++hi)
        for (int lo = 0; lo < n; ++lo)
          inner[g][(r * n + hi) * n + lo] = r > 0 && r < P && hi > 0 && hi < P && lo > 0 && lo < P;
    ioff[g + 1] = ioff[g] + G.nelem * ni;
    aoff[g + 1] = aoff[g] + G.nelem * sc_packed(ni);
    max_loc = std::max<int64_t>(max_loc, G.nelem * n * n * n);
    max_full = std::max<int64_t>(max_full, G.nelem * ni * (int64_t)ni);
  }
  std::vector<int32_t> count(nu, 0);
  std::vector<uint8_t> dir(nu, 0), isb(nu, 0);
  for (int g = 0; g < ng; ++g) {
    const Group& G = s->groups[g];
    const int n3 = (int)inner[g].size();
    for (int64_t i = 0; i < G.nelem * n3; ++i) {
      const int32_t v = m[G.c0 + i], d = l2g_dof(v);
      ++count[d];
      if (v < 0) dir[d] = 1;
      if (!inner[g][i % n3]) isb[d] = 1;
    }
  }
  for (int g = 0; g < ng; ++g) {
    const Group& G = s->groups[g];
    const int n3 = (int)inner[g].size();
    for (int64_t i = 0; i < G.nelem * n3; ++i) {
      const int32_t v = m[G.c0 + i];
      if (inner[g][i % n3] && (v < 0 || count[l2g_dof(v)] != 1))
        return fail(NK_EUNSUPPORTED, "an interior mode's DOF is shared or Dirichlet: the map is not condensable");
    }
  }
  std::vector<int32_t> cpos(nu, -1), bmap;
  for (int64_t d = 0; d < nu; ++d)
    if (isb[d]) {
      cpos[d] = (int32_t)bmap.size();
      bmap.push_back((int32_t)d);
    }
  const int64_t nb = (int64_t)bmap.size();
  std::vector<int32_t> l2gc(nloc), iidx(std::max<int64_t>(ioff[ng], 1));
  std::vector<int8_t> sgn(nloc, 1);
  std::vector<uint8_t> dirc(nb + 1, 0);
  for (int64_t c = 0; c < nb; ++c) dirc[c] = dir[bmap[c]];
  dirc[nb] = 1;
  for (int g = 0; g < ng; ++g) {
    const Group& G = s->groups[g];
    const int n3 = (int)inner[g].size();
    int64_t k = ioff[g];
    for (int64_t i = G.c0; i < G.c0 + G.nelem * n3; ++i) {
      const int32_t d = l2g_dof(m[i]);
      if (inner[g][(i - G.c0) % n3]) {
        l2gc[i] = (int32_t)nb;
        iidx[k++] = d | (l2g_neg(m[i]) ? kL2gNeg : 0);
      } else {
        l2gc[i] = cpos[d];
        sgn[i] = l2g_neg(m[i]) ? -1 : 1;
      }
    }
  }
  CondData* c = new CondData();
  auto bail = [&](nk_status stt) {
    cond_free(c);
    return stt;
  };
  c->nb = nb;
  c->ioff.assign(ioff.begin(), ioff.end());
  int32_t* d_l2g = nullptr;
  int8_t* d_sgn = nullptr;
  uint8_t* d_dir = nullptr;
  if ((e = dmalloc(&d_l2g, nloc)) || (e = dmalloc(&d_sgn, nloc)) || (e = dmalloc(&d_dir, nb + 1)) ||
      (e = hipMemcpyAsync(d_l2g, l2gc.data(), nloc * 4, hipMemcpyHostToDevice, st)) ||
      (e = hipMemcpyAsync(d_sgn, sgn.data(), nloc, hipMemcpyHostToDevice, st)) ||
      (e = hipMemcpyAsync(d_dir, dirc.data(), nb + 1, hipMemcpyHostToDevice, st))) {
    dfree(d_l2g);
    dfree(d_sgn);
    dfree(d_dir);
    return bail(hip_fail(e, "condensation setup"));
  }
  const int64_t eo[2] = {0, E}, dofo[2] = {0, nb + 1};
  const nk_status cs = system_create(&c->bsys, s, 1, eo, dofo, d_l2g, d_sgn, d_dir, y->lam, y->lam0,
                                     st, /*tune=*/false);
  dfree(d_l2g);
  dfree(d_sgn);
  dfree(d_dir);
  if (cs != NK_OK) return bail(cs);
  nk_system z = c->bsys;
  double *cu = nullptr, *yl = nullptr, *afull = nullptr;
  int* d_bad = nullptr;
  auto bail_tmp = [&](hipError_t err) {
    dfree(cu);
    dfree(yl);
    dfree(afull);
    dfree(d_bad);
    return bail(hip_fail(err, "condensation setup"));
  };
  if ((e = dmalloc(&c->bmap, std::max<int64_t>(nb, 1))) ||
      (e = dmalloc(&c->iidx, std::max<int64_t>(ioff[ng], 1))) ||
      (e = dmalloc(&afull, max_full)) || (e = dmalloc(&c->ainv, std::max<int64_t>(aoff[ng], 1))) ||
      (e = dmalloc(&c->t, std::max<int64_t>(ioff[ng], 1))) || (e = dmalloc(&c->zero, z->L.npad)) ||
      (e = dmalloc(&cu, max_loc)) || (e = dmalloc(&yl, max_loc)) || (e = dmalloc(&d_bad, 1)))
    return bail_tmp(e);
  if ((e = hipMemcpyAsync(c->bmap, bmap.data(), nb * 4, hipMemcpyHostToDevice, st)) ||
      (e = hipMemcpyAsync(c->iidx, iidx.data(), ioff[ng] * 4, hipMemcpyHostToDevice, st)) ||
      (e = vec_fill<double>(c->zero, z->L.npad, 0.0, st)) || (e = vec_fill<int32_t>(d_bad, 1, 0, st)))
    return bail_tmp(e);
  c->ops.resize(ng);
  for (int g = 0; g < ng; ++g) {
    const Group& G = s->groups[g];
    const int P = G.P, n3 = (int)inner[g].size(), ni = (P - 1) * (P - 1) * (P - 1);
    const int64_t Eg = G.nelem;
    // H_ii row by row: the local Helmholtz operator on each interior unit vector
    OpArgs a;
    a.op = OP_HELM;
    a.dim = 3;
    a.P = P;
    a.Q = G.Q;
    a.nelem = Eg;
    a.in = cu;
    a.out = yl;
    a.fac = s->fac64 + G.f0;
    a.lam = y->lam ? y->lam + G.e0 : nullptr;
    a.lam0 = y->lam0;
    a.tile = cur_tile(OP_HELM, 3, P, NK_F64);
    a.stream = st;
    if ((e = vec_fill<double>(cu, Eg * n3, 0.0, st))) return bail_tmp(e);
    for (int k = 0; k < ni; ++k) {
      if ((e = sc_unit(P, Eg, cu, k, st)) || (e = launch_op(3, NK_F64, a)) ||
          (e = sc_column(P, Eg, yl, afull, k, st)))
        return bail_tmp(e);
    }
    if ((e = sc_invert(P, Eg, afull, c->ainv + aoff[g], d_bad, st))) return bail_tmp(e);
    CondOp& op = c->ops[g];
    op.P = P;
    op.nelem = Eg;
    op.ainv = c->ainv + aoff[g];
    op.t = c->t + ioff[g];
    op.fac = s->fac64 + G.f0;
    op.fac32 = s->fac32 + G.f0;
    op.lam = z->lam ? z->lam + G.e0 : nullptr;
    op.lam0 = y->lam0;
    op.l2g = z->l2g + G.c0;
  }
  int bad = 0;
  if ((e = hipMemcpyAsync(&bad, d_bad, 4, hipMemcpyDeviceToHost, st)) ||
      (e = hipStreamSynchronize(st)))
    return bail_tmp(e);
  dfree(afull);
  if (bad) {
    dfree(cu);
    dfree(yl);
    dfree(d_bad);
    return bail(fail(NK_EINVAL, "an element's interior block is not positive definite"));
  }
  // Jacobi preconditioner of the boundary system: diag(S) = sum_e diag(S_e),
  // each elemental diagonal probed by the local condensed operator on the
  // boundary unit vectors (all elements of a group at once), replacing the
  // diagonal of the boundary block that the system was created with
  {
    const int64_t npc = z->L.npad;
    double* dS = c->t;   // borrowed when large enough, else a temporary
    double* dS_own = nullptr;
    if (ioff[ng] < npc) {
      if ((e = dmalloc(&dS_own, npc))) return bail_tmp(e);
      dS = dS_own;
    }
    e = vec_fill<double>(dS, npc, 0.0, st);
    for (int g = 0; g < ng && e == hipSuccess; ++g) {
      const Group& G = s->groups[g];
      const int n3 = (int)inner[g].size();
      int prev = -1;
      e = vec_fill<double>(cu, G.nelem * n3, 0.0, st);
      for (int md = 0; md < n3 && e == hipSuccess; ++md) {
        if (inner[g][md]) continue;
        if ((e = sc_unit_mode(G.P, G.nelem, cu, md, prev, st)) ||
            (e = sc_local(c->ops[g], cu, yl, st)) ||
            (e = sc_diag_add(G.P, G.nelem, yl, md, c->ops[g].l2g, dS, st)))
          break;
        prev = md;
      }
    }
    if (e == hipSuccess) e = sc_dinv(npc, dS, z->dinv64, z->dinv32, z->diag, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    dfree(dS_own);
    if (e != hipSuccess) return bail_tmp(e);
  }
  dfree(cu);
  dfree(yl);
  dfree(d_bad);
  z->sc = c->ops.data();
  // the faster of the two fused-kernel variants of each group on this system
  for (int g = 0; g < ng; ++g)
    if ((e = cond_pick_variant(c, g, NK_F64, st))) return bail(hip_fail(e, "condensation setup"));
  y->cond = c;
  return NK_OK;
}

nk_status nk_system_condense(nk_system sys, int64_t* nboundary, int32_t* bmap, double* bdiag,
                             void* stream) {
  if (!sys) return fail(NK_EINVAL, "system is NULL");
  if (!nboundary) return fail(NK_EINVAL, "nboundary is NULL");
  NK_CHECK(check_device());
  hipStream_t st = (hipStream_t)stream;
  NK_CHECK(cond_build(sys, st));
  *nboundary = sys->cond->nb;
  if (bmap) {
    NK_CHECK(check_buf(bmap, (size_t)sys->cond->nb * 4, "bmap"));
    const hipError_t e = hipMemcpyAsync(bmap, sys->cond->bmap, sys->cond->nb * 4,
                                        hipMemcpyDeviceToDevice, st);
    if (e != hipSuccess) return hip_fail(e, "nk_system_condense");
  }
  if (bdiag) {
    NK_CHECK(check_buf(bdiag, (size_t)sys->cond->nb * 8, "bdiag"));
    const hipError_t e = hipMemcpyAsync(bdiag, sys->cond->bsys->diag, sys->cond->nb * 8,
                                        hipMemcpyDeviceToDevice, st);
    if (e != hipSuccess) return hip_fail(e, "nk_system_condense");
  }
  if (bmap || bdiag) {
    const hipError_t e = hipStreamSynchronize(st);
    if (e != hipSuccess) return hip_fail(e, "nk_system_condense");
  }
  return NK_OK;
}

nk_status nk_condensed_apply(nk_system sys, const double* xb, double* yb, void* stream) {
  if (!sys) return fail(NK_EINVAL, "system is NULL");
  if (!sys->cond) return fail(NK_EINVAL, "system has no condensed form (call nk_system_condense)");
  CondData* c = sys->cond;
  nk_system z = c->bsys;
  NK_CHECK(check_buf(xb, (size_t)c->nb * 8, "xb"));
  NK_CHECK(check_buf(yb, (size_t)c->nb * 8, "yb"));
  hipStream_t st = (hipStream_t)stream;
  const int64_t np = z->L.npad;
  hipError_t e;
  if ((e = seg_in(c->nb, np, xb, z->dinv64, z->p, st)) || (e = vec_fill<double>(z->y, np, 0.0, st)) ||
      (e = sys_op(z, NK_F64, z->p, z->y, nullptr, nullptr, st)) ||
      (e = seg_out(c->nb, z->y, yb, st)) || (e = hipStreamSynchronize(st)))
    return hip_fail(e, "condensed apply");
  return NK_OK;
}

// FP64 solve by static condensation with iterative refinement on the full
// system: r = b - A x; the boundary system solves for the correction of r
// (right-hand side g = r_B - sum_e R_e^T H_bi H_ii^{-1} r_i(e)), the interiors
// follow element by element, x is updated and the full true residual
// recomputed; passes repeat until it meets rtol (one pass as a rule).
static nk_status cg_solve_condensed(nk_system y, bool refined, const double* b, double* x,
                                    double rtol, int maxit, nk_solve_info* info, void* stream) {
  const auto t0 = std::chrono::steady_clock::now();
  hipStream_t us = (hipStream_t)stream;
  hipStream_t cs = y->cs;
  hipError_t e = hipSuccess;
  if ((e = hipEventRecord(y->ev, us)) || (e = hipStreamWaitEvent(cs, y->ev, 0)))
    return hip_fail(e, "stream ordering");
  NK_CHECK(cond_build(y, cs));
  CondData* c = y->cond;
  nk_system z = c->bsys;
  if (refined) NK_CHECK(cond_build_f32(c, cs));
  const int kMaxPasses = 4;
  int iters = 0, passes = 0;
  int32_t status = NK_ENOCONV;
  std::vector<double> bb, rr, gg;
  do {
    if ((e = pad_in<double>(1, y->d_dof_off, y->d_pdof_off, y->L, b, y->dinv64, y->b, cs))) break;
    if ((e = pad_in<double>(1, y->d_dof_off, y->d_pdof_off, y->L, x, y->dinv64, y->x, cs))) break;
    if ((e = vec_norm2(y->L, y->b, y->part, y->cnt_aux, y->bb, rtol, nullptr, cs)) ||
        (e = read_sys(y, y->bb, bb)))
      break;
    if ((e = true_residual(y)) || (e = read_sys(y, y->rr_true, rr))) break;
    while (true) {
      if (rel_of(rr[0], bb[0]) <= rtol) {
        status = NK_OK;
        break;
      }
      if (passes == kMaxPasses || iters >= maxit) break;
      ++passes;
      // g: the boundary right-hand side of the residual (the boundary
      // system's work runs on its own stream; y's stream is idle here, as
      // read_sys synchronised it)
      hipStream_t zs = z->cs;
      if ((e = sc_restrict(c->nb, z->L.npad, c->bmap, y->r, z->dinv64, z->b, zs))) break;
      for (size_t g = 0; g < c->ops.size() && e == hipSuccess; ++g)
        if (!(e = sc_ainv(c->ops[g], y->r, c->iidx + c->ioff[g], 0.0, 1.0, -1.0, nullptr, nullptr, zs)))
          e = sc_pass(c->ops[g], 2, c->zero, z->b, nullptr, nullptr, nullptr, zs);
      if (e) break;
      if ((e = vec_fill<double>(z->x, z->L.npad, 0.0, zs)) ||
          (e = vec_norm2(z->L, z->b, z->part, z->cnt_aux, z->bb, rtol, nullptr, zs)) ||
          (e = read_sys(z, z->bb, gg)))
        break;
      // the boundary residual that makes the full one meet rtol
      double rc = gg[0] > 0.0 ? 0.9 * rtol * std::sqrt(bb[0] / gg[0]) : 0.5;
      rc = std::min(rc, 0.5);
      SolveOut so;
      if ((e = solve_padded(z, refined ? NK_SOLVE_F32_REFINED : NK_SOLVE_F64, rc, maxit - iters, so)))
        break;
      iters += so.iters[0];
      if (so.stat[0] == NK_EBREAKDOWN) {
        status = NK_EBREAKDOWN;
        break;
      }
      // interiors: x_i += H_ii^{-1} (r_i - H_ib dx_B); boundary: x_B += dx_B
      for (size_t g = 0; g < c->ops.size() && e == hipSuccess; ++g)
        if (!(e = sc_pass(c->ops[g], 1, z->x, nullptr, nullptr, nullptr, nullptr, zs)))
          e = sc_ainv(c->ops[g], y->r, c->iidx + c->ioff[g], -1.0, 1.0, 1.0, y->x, nullptr, zs);
      if (e || (e = sc_expand_add(c->nb, c->bmap, z->x, y->x, zs)) || (e = hipStreamSynchronize(zs)))
        break;
      if ((e = true_residual(y)) || (e = read_sys(y, y->rr_true, rr))) break;
    }
    if (e) break;
    if ((e = pad_out<double>(1, y->d_dof_off, y->d_pdof_off, y->nuser, y->x, x, cs))) break;
    if ((e = hipEventRecord(y->ev, cs)) || (e = hipStreamWaitEvent(us, y->ev, 0))) break;
    e = hipStreamSynchronize(cs);
  } while (0);
  if (e != hipSuccess) return hip_fail(e, "condensed solve");
  const double ms =
      std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  if (info) {
    info->iters = iters;
    info->outer_iters = passes;
    info->rel_resid = rel_of(rr[0], bb[0]);
    info->solve_ms = ms;
    info->status = status;
  }
  if (status != NK_OK)
    return fail((nk_status)status, status == NK_EBREAKDOWN ? "CG breakdown" : "CG did not converge");
  return NK_OK;
}

nk_status nk_cg_solve(nk_system y, nk_solve_mode mode, const double* b, double* x, double rtol,
                      int maxit, nk_solve_info* info, void* stream) {
  if (!y) return fail(NK_EINVAL, "system is NULL");
  NK_CHECK(check_solve_args(mode, rtol, maxit));
  NK_CHECK(check_buf(b, y->nuser * 8, "b"));
  NK_CHECK(check_buf(x, y->nuser * 8, "x"));
  if (mode == NK_SOLVE_CONDENSED || mode == NK_SOLVE_CONDENSED_F32_REFINED)
    return cg_solve_condensed(y, mode == NK_SOLVE_CONDENSED_F32_REFINED, b, x, rtol, maxit, info,
                              stream);
  const auto t0 = std::chrono::steady_clock::now();
  hipStream_t us = (hipStream_t)stream;
  hipStream_t cs = y->cs;
  const int ns = y->nsys;
  SolveOut o;
  hipError_t e = hipSuccess;
  // order the private stream after the caller's work
  if ((e = hipEventRecord(y->ev, us)) || (e = hipStreamWaitEvent(cs, y->ev, 0)))
    return hip_fail(e, "stream ordering");
  do {
    if ((e = pad_in<double>(ns, y->d_dof_off, y->d_pdof_off, y->L, b, y->dinv64, y->b, cs))) break;
    if ((e = pad_in<double>(ns, y->d_dof_off, y->d_pdof_off, y->L, x, y->dinv64, y->x, cs))) break;
    if ((e = solve_padded(y, mode, rtol, maxit, o))) break;
    if ((e = pad_out<double>(ns, y->d_dof_off, y->d_pdof_off, y->nuser, y->x, x, cs))) break;
    if ((e = hipEventRecord(y->ev, cs)) || (e = hipStreamWaitEvent(us, y->ev, 0))) break;
    e = hipStreamSynchronize(cs);
  } while (0);
  if (e != hipSuccess) return hip_fail(e, "cg solve");
  const double ms =
      std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  nk_status worst = NK_OK;
  for (int i = 0; i < ns; ++i) {
    if (info) fill_info(info + i, o, i, mode, ms);
    if (o.stat[i] != NK_OK && worst == NK_OK) worst = (nk_status)o.stat[i];
  }
  if (worst != NK_OK)
    return fail(worst, worst == NK_EBREAKDOWN ? "CG breakdown" : "CG did not converge");
  return NK_OK;
}

// ------------------------------------------- batched solve of separate systems
// Systems created separately (their own spaces, orders and maps) solved in one
// call.  One-system hexahedral / quadrilateral systems of one (dim, P, Q) form
// a class; a class of two or more is solved as one batched union system
// (their factors, maps, masks and coefficients concatenated into a library-
// owned space and system), so each CG iteration runs one operator launch per
// class with per-system scalars, captured in HIP graphs.  Other systems
// (mixed-order, collapsed shapes, already batched) run as their own lanes.
// Lanes run concurrently, each on its own private stream.  Unions are cached
// by their member list (at most kMaxUnions, least recently used dropped) and
// freed when a member is destroyed.
namespace {
struct UnionLane {
  std::vector<nk_system> members;
  nk_space space = nullptr;
  nk_system sys = nullptr;
};
std::mutex g_union_mu;
std::vector<UnionLane*> g_unions;   // least recently used first
constexpr size_t kMaxUnions = 4;
}  // namespace

static void union_free(UnionLane* u) {
  if (!u) return;
  system_free(u->sys);
  space_free(u->space);
  delete u;
}

// Drop every cached union that holds system y (called on destroy).
static void union_forget(nk_system y) {
  std::lock_guard<std::mutex> lk(g_union_mu);
  for (size_t i = 0; i < g_unions.size();) {
    UnionLane* u = g_unions[i];
    if (std::find(u->members.begin(), u->members.end(), y) != u->members.end()) {
      union_free(u);
      g_unions.erase(g_unions.begin() + i);
    } else {
      ++i;
    }
  }
}

static bool union_member_ok(nk_system y) {
  return y->nsys == 1 && y->space->shape == 0 && y->space->groups.size() == 1;
}

// Build the union of members (same dim, P, Q; one system each) on stream st.
static nk_status union_build(const std::vector<nk_system>& mem, hipStream_t st, UnionLane** out) {
  const int m = (int)mem.size();
  const nk_space s0 = mem[0]->space;
  const Group& G0 = s0->groups[0];
  std::vector<int64_t> eoff(m + 1, 0), doff(m + 1, 0), coff(m + 1, 0);
  int64_t nfac = 0;
  bool per_elem_lam = false;
  for (int k = 0; k < m; ++k) {
    const nk_space sk = mem[k]->space;
    eoff[k + 1] = eoff[k] + sk->nelem;
    doff[k + 1] = doff[k] + mem[k]->nuser;
    coff[k + 1] = coff[k] + sk->ncoeff;
    nfac += sk->nfac;
    if (mem[k]->lam || mem[k]->lam0 != mem[0]->lam0) per_elem_lam = true;
  }
  if (doff[m] >= ((int64_t)1 << 30)) return fail(NK_EINVAL, "batched systems: too many global DOFs");
  UnionLane* u = new UnionLane();
  u->members = mem;
  nk_space s = new nk_space_s();
  u->space = s;
  s->dim = s0->dim;
  s->shape = 0;
  s->device = s0->device;
  Group G;
  G.P = G0.P;
  G.Q = G0.Q;
  G.n = G0.n;
  G.nelem = eoff[m];
  s->groups.push_back(G);
  s->nelem = eoff[m];
  s->ncoeff = coff[m];
  s->npoint = eoff[m] * ipow(G.Q, s->dim);
  s->nfac = nfac;
  int32_t* l2g = nullptr;
  int8_t* sign = nullptr;
  uint8_t* dir = nullptr;
  double* lam = nullptr;
  auto done = [&](nk_status stt) {
    dfree(l2g);
    dfree(sign);
    dfree(dir);
    dfree(lam);
    if (stt != NK_OK) union_free(u);
    return stt;
  };
  hipError_t e;
  if ((e = dmalloc(&s->fac64, std::max<int64_t>(nfac, 1))) ||
      (e = dmalloc(&s->fac32, std::max<int64_t>(nfac, 1))) ||
      (e = dmalloc(&l2g, std::max<int64_t>(coff[m], 1))) ||
      (e = dmalloc(&sign, std::max<int64_t>(coff[m], 1))) ||
      (e = dmalloc(&dir, std::max<int64_t>((doff[m] + 3) / 4 * 4, 4))) ||
      (per_elem_lam && (e = dmalloc(&lam, std::max<int64_t>(eoff[m], 1)))))
    return done(hip_fail(e, "hipMalloc"));
  do {
    if ((e = vec_fill<int32_t>((int32_t*)dir, (doff[m] + 3) / 4, 0, st))) break;
    int64_t f = 0;
    for (int k = 0; k < m && e == hipSuccess; ++k) {
      const nk_space sk = mem[k]->space;
      if (sk->nfac > 0 &&
          ((e = hipMemcpyAsync(s->fac64 + f, sk->fac64, sk->nfac * 8, hipMemcpyDeviceToDevice, st)) ||
           (e = hipMemcpyAsync(s->fac32 + f, sk->fac32, sk->nfac * 4, hipMemcpyDeviceToDevice, st))))
        break;
      f += sk->nfac;
      if ((e = decode_l2g(sk->ncoeff, mem[k]->l2g, doff[k], l2g + coff[k], sign + coff[k], dir, st)))
        break;
      if (per_elem_lam && sk->nelem > 0) {
        if (mem[k]->lam)
          e = hipMemcpyAsync(lam + eoff[k], mem[k]->lam, sk->nelem * 8, hipMemcpyDeviceToDevice, st);
        else
          e = vec_fill<double>(lam + eoff[k], sk->nelem, mem[k]->lam0, st);
      }
    }
    if (e == hipSuccess) e = hipStreamSynchronize(st);
  } while (0);
  if (e != hipSuccess) return done(hip_fail(e, "batched systems setup"));
  const nk_status cs = system_create(&u->sys, s, m, eoff.data(), doff.data(), l2g, sign, dir, lam,
                                     mem[0]->lam0, st);
  if (cs != NK_OK) return done(cs);
  *out = u;
  return done(NK_OK);
}

// The cached union of exactly these members, built if absent.
static nk_status union_get(const std::vector<nk_system>& mem, hipStream_t st, UnionLane** out) {
  std::lock_guard<std::mutex> lk(g_union_mu);
  for (size_t i = 0; i < g_unions.size(); ++i) {
    if (g_unions[i]->members == mem) {
      UnionLane* u = g_unions[i];
      g_unions.erase(g_unions.begin() + i);
      g_unions.push_back(u);
      *out = u;
      return NK_OK;
    }
  }
  UnionLane* u = nullptr;
  NK_CHECK(union_build(mem, st, &u));
  if (g_unions.size() >= kMaxUnions) {
    union_free(g_unions.front());
    g_unions.erase(g_unions.begin());
  }
  g_unions.push_back(u);
  *out = u;
  return NK_OK;
}

namespace {
struct Lane {
  nk_system sys = nullptr;    // what is solved: a union or one caller system
  bool is_union = false;
  std::vector<int> idx;       // caller indices, in the system's order
  SolveOut out;
  hipError_t err = hipSuccess;
};
}  // namespace

static void run_lane(Lane& L, int dev, nk_solve_mode mode, const double* const* b, double* const* x,
                     double rtol, int maxit) {
  nk_system y = L.sys;
  hipStream_t cs = y->cs;
  hipError_t e = hipSetDevice(dev);
  do {
    if (e) break;
    if (L.is_union) {
      for (int k = 0; k < y->nsys && e == hipSuccess; ++k) {
        const int64_t n = y->dof_off[k + 1] - y->dof_off[k];
        const int64_t p0 = y->pdof_off[k], np = y->pdof_off[k + 1] - p0;
        if ((e = seg_in(n, np, b[L.idx[k]], y->dinv64 + p0, y->b + p0, cs))) break;
        e = seg_in(n, np, x[L.idx[k]], y->dinv64 + p0, y->x + p0, cs);
      }
    } else {
      const int j = L.idx[0];
      if ((e = pad_in<double>(y->nsys, y->d_dof_off, y->d_pdof_off, y->L, b[j], y->dinv64, y->b, cs)))
        break;
      e = pad_in<double>(y->nsys, y->d_dof_off, y->d_pdof_off, y->L, x[j], y->dinv64, y->x, cs);
    }
    if (e) break;
    if ((e = solve_padded(y, mode, rtol, maxit, L.out))) break;
    if (L.is_union) {
      for (int k = 0; k < y->nsys && e == hipSuccess; ++k)
        e = seg_out(y->dof_off[k + 1] - y->dof_off[k], y->x + y->pdof_off[k], x[L.idx[k]], cs);
    } else {
      e = pad_out<double>(y->nsys, y->d_dof_off, y->d_pdof_off, y->nuser, y->x, x[L.idx[0]], cs);
    }
    if (e) break;
    e = hipStreamSynchronize(cs);
  } while (0);
  L.err = e;
}

nk_status nk_cg_solve_batched(nk_system* sys, int nsys, nk_solve_mode mode, const double* const* b,
                              double* const* x, double rtol, int maxit, nk_solve_info* info,
                              void* stream) {
  if (!sys || !b || !x) return fail(NK_EINVAL, "sys, b and x must be non-NULL");
  if (nsys < 1) return fail(NK_EINVAL, "nsys must be >= 1");
  NK_CHECK(check_solve_args(mode, rtol, maxit));
  if (mode == NK_SOLVE_CONDENSED || mode == NK_SOLVE_CONDENSED_F32_REFINED)
    return fail(NK_EUNSUPPORTED, "the condensed modes solve one system per nk_cg_solve call");
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  for (int i = 0; i < nsys; ++i) {
    if (!sys[i]) return fail(NK_EINVAL, "system " + std::to_string(i) + " is NULL");
    if (sys[i]->device != dev)
      return fail(NK_EINVAL, "system " + std::to_string(i) + " lives on another device");
    for (int j = 0; j < i; ++j)
      if (sys[j] == sys[i]) return fail(NK_EINVAL, "a system appears twice in the batch");
    NK_CHECK(check_buf(b[i], sys[i]->nuser * 8, "b"));
    NK_CHECK(check_buf(x[i], sys[i]->nuser * 8, "x"));
  }
  const auto t0 = std::chrono::steady_clock::now();
  hipStream_t us = (hipStream_t)stream;
  // classes of union-able systems, in caller order
  std::vector<Lane> lanes;
  std::map<std::tuple<int, int, int>, std::vector<int>> cls;
  std::vector<std::tuple<int, int, int>> cls_order;
  for (int i = 0; i < nsys; ++i) {
    if (union_member_ok(sys[i])) {
      const Group& G = sys[i]->space->groups[0];
      const auto key = std::make_tuple(sys[i]->space->dim, G.P, G.Q);
      if (!cls.count(key)) cls_order.push_back(key);
      cls[key].push_back(i);
    } else {
      Lane L;
      L.sys = sys[i];
      L.idx = {i};
      lanes.push_back(std::move(L));
    }
  }
  // a union's setup runs on the caller's stream after the caller's work
  for (const auto& key : cls_order) {
    const std::vector<int>& ids = cls[key];
    Lane L;
    L.idx = ids;
    if (ids.size() == 1) {
      L.sys = sys[ids[0]];
    } else {
      std::vector<nk_system> mem;
      for (int i : ids) mem.push_back(sys[i]);
      UnionLane* u = nullptr;
      NK_CHECK(union_get(mem, us, &u));
      L.sys = u->sys;
      L.is_union = true;
    }
    lanes.push_back(std::move(L));
  }
  // order every lane's private stream after the caller's work
  for (Lane& L : lanes)
    if ((e = hipEventRecord(L.sys->ev, us)) || (e = hipStreamWaitEvent(L.sys->cs, L.sys->ev, 0)))
      return hip_fail(e, "stream ordering");
  if (lanes.size() == 1) {
    run_lane(lanes[0], dev, mode, b, x, rtol, maxit);
  } else {
    std::vector<std::thread> th;
    for (Lane& L : lanes)
      th.emplace_back(run_lane, std::ref(L), dev, mode, b, x, rtol, maxit);
    for (std::thread& t : th) t.join();
  }
  for (Lane& L : lanes)
    if (L.err != hipSuccess) return hip_fail(L.err, "batched cg solve");
  for (Lane& L : lanes)
    if ((e = hipEventRecord(L.sys->ev, L.sys->cs)) || (e = hipStreamWaitEvent(us, L.sys->ev, 0)))
      return hip_fail(e, "stream ordering");
  const double ms =
      std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  nk_status worst = NK_OK;
  for (Lane& L : lanes) {
    for (int32_t st : L.out.stat)
      if (st != NK_OK && worst == NK_OK) worst = (nk_status)st;
    if (!info) continue;
    if (L.is_union || L.sys->nsys == 1) {
      for (size_t k = 0; k < L.idx.size(); ++k) fill_info(info + L.idx[k], L.out, (int)k, mode, ms);
    } else {
      // a caller system that is itself batched: its entry is the sub-system
      // with the largest residual, with the worst status of all of them
      int kw = 0;
      for (int k = 1; k < L.sys->nsys; ++k)
        if (rel_of(L.out.rr[k], L.out.bb[k]) > rel_of(L.out.rr[kw], L.out.bb[kw])) kw = k;
      fill_info(info + L.idx[0], L.out, kw, mode, ms);
      for (int k = 0; k < L.sys->nsys; ++k) {
        info[L.idx[0]].iters = std::max(info[L.idx[0]].iters, L.out.iters[k]);
        if (L.out.stat[k] != NK_OK) info[L.idx[0]].status = L.out.stat[k];
      }
    }
  }
  if (worst != NK_OK)
    return fail(worst, worst == NK_EBREAKDOWN ? "CG breakdown" : "CG did not converge");
  return NK_OK;
}

// --------------------------------------------------------------- autotune
static std::mutex g_tune_mu;

static std::string device_name() {
  hipDeviceProp_t p;
  int dev = 0;
  (void)hipGetDevice(&dev);
  if (hipGetDeviceProperties(&p, dev) != hipSuccess) return "unknown";
  std::string n = p.gcnArchName;
  for (char& c : n)
    if (c == ' ' || c == ':') c = '_';
  return n;
}

static bool cache_lookup(const std::string& key, int* tile) {
  const char* path = std::getenv("NK_AUTOTUNE_CACHE");
  if (!path) return false;
  std::ifstream f(path);
  std::string line, k;
  int t = -1;
  bool found = false;
  while (std::getline(f, line)) {
    std::istringstream is(line);
    if (is >> k >> t && k == key) {
      *tile = t;
      found = true;
    }
  }
  return found;
}

static void cache_store(const std::string& key, int tile, double us) {
  const char* path = std::getenv("NK_AUTOTUNE_CACHE");
  if (!path) return;
  std::ofstream f(path, std::ios::app);
  f << key << " " << tile << " " << us << "\n";
}

// Tile of a system's assembled operator for order group g: the caller's
// explicit Helmholtz choice if there is one, else the fastest candidate timed
// on this system's own operator (2 warm-up + 4 timed applications each), remembered per
// process (and in NK_AUTOTUNE_CACHE) by order and dtype.
static int tune_asm_tile(nk_system y, nk_dtype t, int g, hipStream_t st) {
  nk_space s = y->space;
  const Group& G = s->groups[g];
  if (s->shape != 0) return 0;   // collapsed-shape kernels have one launch shape
  const int fallback = cur_tile(OP_HELM_ASM, s->dim, G.P, t);
  const int nt = tile_count(OP_HELM_ASM, s->dim, G.P);
  if (nt <= 1 || G.nelem == 0 || g_tile_forced[s->dim - 2][G.P][t].load()) return fallback;
  static std::map<std::string, int> memo;
  std::lock_guard<std::mutex> lk(g_tune_mu);
  const std::string key = "asm_d" + std::to_string(s->dim) + "_P" + std::to_string(G.P) + "_Q" +
                          std::to_string(G.Q) + "_" + (t == NK_F64 ? "f64" : "f32") + "_E2^" +
                          std::to_string((int)std::log2((double)G.nelem)) + "_" + device_name();
  auto it = memo.find(key);
  if (it != memo.end()) return it->second;
  int best = fallback;
  if (!cache_lookup(key, &best)) {
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
      if (e0) (void)hipEventDestroy(e0);
      return fallback;
    }
    const void* x = t == NK_F64 ? (const void*)y->p : (const void*)y->p32;
    void* o = t == NK_F64 ? (void*)y->y : (void*)y->y32;
    double best_us = 1e30;
    for (int k = 0; k < nt; ++k) {
      hipError_t e = hipSuccess;
      for (int w = 0; w < 2 && e == hipSuccess; ++w) e = sys_op_group(y, t, g, x, o, nullptr, nullptr, k, st);
      (void)hipEventRecord(e0, st);
      for (int r = 0; r < 4 && e == hipSuccess; ++r) e = sys_op_group(y, t, g, x, o, nullptr, nullptr, k, st);
      (void)hipEventRecord(e1, st);
      (void)hipEventSynchronize(e1);
      if (e != hipSuccess) {
        best = fallback;
        best_us = -1.0;
        break;
      }
      float ms = 0.f;
      (void)hipEventElapsedTime(&ms, e0, e1);
      if (250.0 * ms < best_us) {
        best_us = 250.0 * ms;
        best = k;
      }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (best_us < 0) return fallback;
    cache_store(key, best, best_us);
  }
  memo[key] = best;
  return best;
}

nk_status nk_autotune(nk_space s, int op_mask, void* stream) {
  if (!s) return fail(NK_EINVAL, "space is NULL");
  if (s->shape != 0) return NK_OK;   // triangles have a single launch shape per order
  NK_CHECK(check_device());
  std::lock_guard<std::mutex> lk(g_tune_mu);
  hipStream_t st = (hipStream_t)stream;
  const std::string dev = device_name();
  // scratch operands large enough for every op of the space
  const int64_t big = std::max(s->ncoeff, s->npoint);
  double *a = nullptr, *b = nullptr;
  hipError_t e;
  if ((e = dmalloc(&a, std::max<int64_t>(big, 1))) || (e = dmalloc(&b, std::max<int64_t>(big, 1)))) {
    dfree(a);
    dfree(b);
    return hip_fail(e, "hipMalloc");
  }
  (void)vec_fill<double>(a, big, 0.5, st);
  hipEvent_t e0, e1;
  (void)hipEventCreate(&e0);
  (void)hipEventCreate(&e1);
  nk_status result = NK_OK;
  for (const Group& G : s->groups) {
    if (G.nelem == 0) continue;
    for (int op = 0; op <= OP_HELM && result == NK_OK; ++op) {
      if (!(op_mask >> op & 1)) continue;
      for (nk_dtype t : {NK_F64, NK_F32}) {
        const int nt = tile_count(op, s->dim, G.P);
        std::string key = "op" + std::to_string(op) + "_d" + std::to_string(s->dim) + "_P" +
                          std::to_string(G.P) + "_Q" + std::to_string(G.Q) + "_" +
                          (t == NK_F64 ? "f64" : "f32") + "_" + dev;
        int best = 0;
        if (nt > 1 && !cache_lookup(key, &best)) {
          // two interleaved passes over the candidates, each candidate's
          // best pass kept, so a clock or thermal drift during one pass does
          // not decide between candidates a few per cent apart
          std::vector<double> us_k(nt, 1e30);
          for (int pass = 0; pass < 2 && result == NK_OK; ++pass)
          for (int k = 0; k < nt; ++k) {
            OpArgs o;
            o.op = op;
            o.dim = s->dim;
            o.P = G.P;
            o.Q = G.Q;
            o.nelem = G.nelem;
            o.in = a;
            o.out = b;
            o.fac = t == NK_F64 ? (const void*)(s->fac64 + G.f0) : (const void*)(s->fac32 + G.f0);
            o.lam0 = 1.0;
            o.tile = k;
            o.stream = st;
            for (int w = 0; w < 2; ++w) e = launch_op(s->dim, t, o);
            const int reps = 5;
            (void)hipEventRecord(e0, st);
            for (int r = 0; r < reps && e == hipSuccess; ++r) e = launch_op(s->dim, t, o);
            (void)hipEventRecord(e1, st);
            (void)hipEventSynchronize(e1);
            if (e != hipSuccess) {
              result = hip_fail(e, "autotune launch");
              break;
            }
            float ms = 0.f;
            (void)hipEventElapsedTime(&ms, e0, e1);
            us_k[k] = std::min(us_k[k], 1000.0 * ms / reps);
          }
          for (int k = 1; k < nt; ++k)
            if (us_k[k] < us_k[best]) best = k;
          if (result == NK_OK) cache_store(key, best, us_k[best]);
        }
        if (result == NK_OK) {
          (void)cur_tile(op, s->dim, G.P, t);  // runs the one-time default initialisation
          g_tile[op][s->dim - 2][G.P][t].store(best);
        }
      }
    }
  }
  // mixed-order spaces: time the evaluation strategies of the Helmholtz
  // operator on the whole space and keep the fastest (per dtype)
  if (result == NK_OK && s->groups.size() > 1 && (op_mask >> OP_HELM & 1)) {
    for (nk_dtype t : {NK_F64, NK_F32}) {
      double best_us = 1e30;
      int best = VARP_PERSISTENT;
      for (int k = 0; k < VARP_COUNT && result == NK_OK; ++k) {
        s->varp_strategy[t] = k;
        nk_status r2 = NK_OK;
        for (int w = 0; w < 2 && r2 == NK_OK; ++w)
          r2 = space_op(s, OP_HELM, t, a, b, nullptr, 1.0, nullptr, st);
        const int reps = 5;
        (void)hipEventRecord(e0, st);
        for (int r = 0; r < reps && r2 == NK_OK; ++r)
          r2 = space_op(s, OP_HELM, t, a, b, nullptr, 1.0, nullptr, st);
        (void)hipEventRecord(e1, st);
        (void)hipEventSynchronize(e1);
        if (r2 != NK_OK) {
          result = r2;
          break;
        }
        float ms = 0.f;
        (void)hipEventElapsedTime(&ms, e0, e1);
        if (1000.0 * ms / reps < best_us) {
          best_us = 1000.0 * ms / reps;
          best = k;
        }
      }
      s->varp_strategy[t] = best;
    }
  }
  (void)hipStreamSynchronize(st);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  dfree(a);
  dfree(b);
  return result;
}

nk_status nk_set_tile_config(int op, int dim, int P, nk_dtype t, int tile) {
  if (op < 0 || op > OP_HELM || (dim != 2 && dim != 3) || P < kMinP || P > kMaxP ||
      (t != NK_F64 && t != NK_F32))
    return fail(NK_EINVAL, "bad operator, dimension, order or dtype");
  if (tile < 0 || tile >= tile_count(op, dim, P)) return fail(NK_EINVAL, "tile index out of range");
  (void)cur_tile(op, dim, P, t);
  g_tile[op][dim - 2][P][t].store(tile);
  if (op == OP_HELM) g_tile_forced[dim - 2][P][t].store(true);
  return NK_OK;
}

int nk_tile_count(int op, int dim, int P) {
  if (op < 0 || op >= OP_COUNT || (dim != 2 && dim != 3)) return 0;
  return tile_count(op, dim, P);
}

const char* nk_tile_config(int op, int dim, int P, nk_dtype t) {
  if (op < 0 || op >= OP_COUNT || (dim != 2 && dim != 3) || P < kMinP || P > kMaxP) return "";
  return tile_name(op, dim, P, cur_tile(op, dim, P, t));
}
