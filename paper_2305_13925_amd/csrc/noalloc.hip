// The batched precoder path for callers that cannot allocate device memory
// (code under HIP graph capture, serving loops that forbid hipMalloc): the
// workspace of one call (A, diag(H^H H), X, the solver's per-workgroup power
// partials and statuses) lives in a fixed device array of the library instead
// of the session's arena. Every call on one GPU shares that GPU's array, so
// calls that overlap on one GPU race; nothing in it has to start at zero (each
// kernel writes every workspace entry it later reads).
#include <hip/hip_runtime.h>

#include <mutex>

#include "../../include/jacpcg.h"
#include "common.hpp"
#include "session.hpp"

namespace {

constexpr size_t kScratchBytes = (size_t)96 << 20;
constexpr int kMaxDevices = 64;

// Device-side workspace; its host-side name is only a handle for
// hipGetSymbolAddress and is never passed to a kernel or copy.
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_mu;
void* g_ptr[kMaxDevices];            // device address of `scratch` on each device
hipError_t g_err[kMaxDevices];       // result of the look-up on each device
bool g_done[kMaxDevices];

}  // namespace

namespace jacpcg {

size_t noalloc_scratch_bytes() { return kScratchBytes; }

// Look up the array's device address once per device; the device must be
// current. Called at session creation.
hipError_t noalloc_setup(int device) {
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_mu);
  if (g_done[device]) return g_err[device];
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess) (void)hipGetLastError();
  g_ptr[device] = e == hipSuccess ? p : nullptr;
  g_err[device] = e;
  g_done[device] = true;
  return e;
}

// Bytes of the array one call needs: the same buffers as the batched path,
// each 256-byte aligned.
size_t noalloc_need(int batch, int K) {
  Workspace ws;
  const int ncb = (K + 31) / 32;
  ws.take<float2>((size_t)batch * K * K);  // A
  ws.take<float>((size_t)batch * K);       // diag(H^H H)
  ws.take<float2>((size_t)batch * K * K);  // X
  ws.take<float>((size_t)batch * ncb);     // power partials
  ws.take<int32_t>((size_t)batch * ncb);   // workgroup statuses
  return ws.bytes;
}

// Gram -> persistent Jacobi-PCG (B = I_K) -> precoder, with every workspace
// buffer carved from the device's array. Arguments are validated by the
// caller; the sizes fit (noalloc_need <= noalloc_scratch_bytes()).
int run_rzf_noalloc(jacpcg_session* s, hipStream_t st, int batch, int M, int K, const float2* H, int64_t ldh,
                    int64_t stride_h, double xi, double power, double tol, int max_iter, int gram_prec,
                    bool precond_none, bool split_epilogue, float2* W, int64_t ldw, int64_t stride_w,
                    int32_t* status) {
  if (s->device < 0 || s->device >= kMaxDevices) return set_error(JACPCG_E_NO_DEVICE, "device out of range");
  const PhaseRange range("rzf_precoder_noalloc");
  char* base = nullptr;
  {
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_done[s->device]) return set_error(JACPCG_E_HIP, "scratch array not set up on this device");
    if (g_err[s->device] != hipSuccess) {
      const std::string m = std::string("hipGetSymbolAddress(scratch) failed: ") + hipGetErrorString(g_err[s->device]);
      return set_error(JACPCG_E_HIP, m.c_str());
    }
    base = static_cast<char*>(g_ptr[s->device]);
  }
  const int ncb = (K + 31) / 32;
  const size_t KK = (size_t)K * K;
  Workspace ws;
  const size_t oA = ws.take<float2>((size_t)batch * KK);
  const size_t oG = ws.take<float>((size_t)batch * K);
  const size_t oX = ws.take<float2>((size_t)batch * KK);
  const size_t oF = ws.take<float>((size_t)batch * ncb);
  const size_t oWG = ws.take<int32_t>((size_t)batch * ncb);
  if (ws.bytes > kScratchBytes) return set_error(JACPCG_E_INVALID_ARG, "batch does not fit the scratch array");
  float2* A = reinterpret_cast<float2*>(base + oA);
  float* gdiag = reinterpret_cast<float*>(base + oG);
  float2* X = reinterpret_cast<float2*>(base + oX);
  float* fpart = reinterpret_cast<float*>(base + oF);
  int32_t* wgs = reinterpret_cast<int32_t*>(base + oWG);

  GramLaunch g{};
  g.H = H;
  g.ldh = ldh;
  g.stride_h = stride_h;
  g.batch = batch;
  g.M = M;
  g.K = K;
  g.xi = (float)xi;
  g.A = A;
  g.lda = K;
  g.stride_a = (int64_t)KK;
  g.gdiag = gdiag;
  g.precision = gram_prec;
  g.m_split = s->tuner.gram_waves(M, K, gram_prec);
  hipError_t e = launch_gram(g, st);
  if (e == hipErrorNotSupported) return set_error(JACPCG_E_UNSUPPORTED, "Gram precision not available");
  if (e != hipSuccess) return set_error(JACPCG_E_HIP, hipGetErrorString(e));

  PcgLaunch p{};
  p.A = A;
  p.lda = K;
  p.stride_a = (int64_t)KK;
  p.X = X;
  p.ldx = K;
  p.stride_x = (int64_t)KK;
  p.batch = batch;
  p.K = K;
  p.nrhs = K;
  p.tol = (float)tol;
  p.max_iter = max_iter;
  p.precond_none = precond_none;
  p.wg_status = wgs;
  p.gdiag = gdiag;
  p.fpart = fpart;
  p.a_source = s->tuner.pcg_a_source(K);
  e = launch_pcg(p, st, nullptr);
  if (e != hipSuccess) return set_error(JACPCG_E_HIP, hipGetErrorString(e));

  PrecoderLaunch E{};
  E.H = H;
  E.ldh = ldh;
  E.stride_h = stride_h;
  E.X = X;
  E.ldx = K;
  E.stride_x = (int64_t)KK;
  E.W = W;
  E.ldw = ldw;
  E.stride_w = stride_w;
  E.batch = batch;
  E.M = M;
  E.K = K;
  E.nrhs = K;
  E.fpart = fpart;
  E.ncb = ncb;
  E.power = (float)power;
  E.wg_status = wgs;
  E.status = status;
  E.split = split_epilogue ? 3 : 0;
  E.nj = s->tuner.precoder_nj(M, K, E.split);
  E.mtiles = s->tuner.precoder_mtiles(M, K, E.split);
  e = launch_precoder(E, st);
  if (e != hipSuccess) return set_error(JACPCG_E_HIP, hipGetErrorString(e));
  return JACPCG_OK;
}

}  // namespace jacpcg
