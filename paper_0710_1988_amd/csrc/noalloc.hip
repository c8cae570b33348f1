// Operator apply for callers that cannot allocate device memory (code under HIP graph capture,
// tight serving loops): the packed links and vectors live in one static device array instead of
// the context's workspace pool.  Each GPU holds its own copy of the array for the life of the
// process; every call on a GPU uses the same copy, so calls that overlap on one GPU race.
#include <cstring>
#include <mutex>

#include "ctx.h"
#include "kernels.h"

namespace dbq {

namespace {

constexpr size_t SCRATCH_BYTES = size_t(64) << 20;  // 64 MiB per GPU
static __device__ __align__(256) unsigned char scratch[SCRATCH_BYTES];

constexpr int MAX_DEVICES = 64;
void* scratch_of_device[MAX_DEVICES] = {};
std::mutex scratch_mutex;

size_t round256(size_t b) { return (b + 255) & ~size_t(255); }

}  // namespace

size_t noalloc_scratch_bytes() { return SCRATCH_BYTES; }

// Device address of the current device's copy of the static scratch array, looked up once per
// device (with that device current) and kept: in host code the array's name is only a host-side
// stand-in, never a device address.
void* noalloc_scratch(int device) {
  DBQ_CHECK(device >= 0 && device < MAX_DEVICES, "device index out of range");
  std::lock_guard<std::mutex> lock(scratch_mutex);
  if (!scratch_of_device[device]) {
    void* p = nullptr;
    DBQ_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    DBQ_CHECK(p != nullptr, "no device address for the static scratch array");
    scratch_of_device[device] = p;
  }
  return scratch_of_device[device];
}

void apply_operator_noalloc(dbq_ctx* c, const dbq_operator* o, const void* in, void* out,
                            int nrhs, int dagger, int prec) {
  DBQ_CHECK(o != nullptr && in && out, "null argument");
  DBQ_CHECK(in != out, "in and out must not alias");
  DBQ_CHECK(nrhs >= 1, "nrhs must be >= 1");
  DBQ_CHECK(prec == DBQ_FP64 || prec == DBQ_MIXED, "bad precision");
  long long V = 1;
  for (int i = 0; i < 4; ++i) {
    DBQ_CHECK(o->L[i] >= 2 && o->L[i] % 2 == 0, "lattice extents must be even and >= 2");
    V *= o->L[i];
  }
  DBQ_CHECK(V <= (1ll << 26), "lattice too large (V > 2^26)");
  DBQ_CHECK(o->links != nullptr, "null links");
  DBQ_CHECK(o->schur == 0, "the allocation-free apply takes the full operator only (schur = 0)");
  DBQ_CHECK(o->pad == 0, "operator pad field must be 0");
  const bool f32 = prec == DBQ_MIXED;
  // packed links, then the packed input and output vectors
  const size_t lbytes = round256(size_t(V) * (f32 ? 12 * sizeof(float4) : 36 * sizeof(double2)));
  const size_t vbytes =
      round256(size_t(V) * nrhs * (f32 ? 6 * sizeof(float4) : 12 * sizeof(double2)));
  const size_t need = lbytes + 2 * vbytes;
  if (need > SCRATCH_BYTES)
    throw Error(DBQ_EINVAL, "allocation-free apply needs " + std::to_string(need) +
                                " bytes of scratch, more than its " +
                                std::to_string(SCRATCH_BYTES) + " (fewer rhs or a smaller lattice)");
  if (!c->scratch) c->scratch = noalloc_scratch(c->device);
  char* base = static_cast<char*>(c->scratch);
  const Geom g = make_geom(o->L);
  DsBatch b;
  std::memset(&b, 0, sizeof(b));
  b.nlat = 1;
  b.nrhs_total = nrhs;
  b.pstride = 1;
  DsLat& L = b.lat[0];
  L.g = g;
  L.links = base;
  L.in = base + lbytes;
  L.out = base + lbytes + vbytes;
  L.nrhs = nrhs;
  L.kappa = o->kappa;
  L.mu = o->mu;
  if (f32) {
    pack_links_f32(c->stream, g, o->links, (float4*)base);
    pack_spinor_f32(c->stream, g, in, (float4*)(base + lbytes), nrhs);
    // the LDS tile kernel with every rhs per block, tiles visited region by region
    b.torder = 1;
    launch_dslash_f32(c->stream, b, dagger, EPI_NONE, nullptr, nullptr, 0, 0);
    unpack_spinor_f32(c->stream, g, (const float4*)(base + lbytes + vbytes), out, nrhs);
  } else {
    pack_links_f64(c->stream, g, o->links, (double2*)base);
    pack_spinor_f64(c->stream, g, in, (double2*)(base + lbytes), nrhs);
    launch_dslash_f64(c->stream, b, dagger, EPI_NONE, nullptr, nullptr, 1, 0);
    unpack_spinor_f64(c->stream, g, (const double2*)(base + lbytes + vbytes), out, nrhs);
  }
}

}  // namespace dbq
