// Host emulation of the HIP runtime calls the library makes, for running the
// library's host logic on a machine without a GPU under AddressSanitizer.
//
// Device memory is host memory.  Copies and fills are asynchronous as on the
// real runtime: each is queued on its stream and only performed when that
// stream (or an event recorded on it, or a stream that waited on such an
// event) is synchronised.  Until then the host destination of a
// device-to-host copy is poisoned (a host read before the synchronisation is
// reported), and the host source of a host-to-device copy is snapshotted (a
// host write before the copy runs is reported; a source that is freed first is
// reported by AddressSanitizer when the copy runs).  Stream capture records the
// copies and fills of every stream in the capture (the origin and the streams
// forked from it through events) as graph nodes, replayed at every graph
// launch; kernel launches are checked (grid and block within the hardware
// limits, LDS within 64 KiB), counted and, when captured, counted per graph.
// A capture that ends with a forked stream not joined back, or a synchronous
// call on a capturing stream, is reported as an error.  The code-object
// symbols that host-only objects reference are defined by a generated file
// next to this one.
#include <sanitizer/asan_interface.h>

#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <set>
#include <vector>

#include <hip/hip_runtime_api.h>

namespace {

struct Op {
  long long seq;
  int kind;  // 0 copy, 1 fill
  void* dst;
  const void* src;
  size_t n;
  int value;
  hipMemcpyKind dir;
  std::vector<char> snap;  // host source at enqueue (host-to-device)
};

struct Stream {
  std::vector<Op> q;
  struct Dep {
    Stream* on;
    long long upto;  // the waited event's position on `on`
    long long at;    // position of the wait on this stream
  };
  std::vector<Dep> deps;
  bool capturing = false;
  struct Graph* graph = nullptr;
  long long last_join_seq = -1;  // seq of this stream's last event joined back
  long long last_op_seq = -1;
};

struct Event {
  Stream* s = nullptr;
  long long seq = -1;
};

struct Graph {
  std::vector<Op> nodes;
  long launches = 0;
  std::set<Stream*> members;
  Stream* origin = nullptr;
};

long long g_seq = 0;
Stream g_null;  // the legacy default stream
long g_errors = 0;
// every stream ever created (destroyed ones stay allocated, so events and
// dependencies that name them stay valid, as on the runtime)
// (held through a pointer that is never freed, so they stay reachable)
std::vector<Stream*>& g_streams = *new std::vector<Stream*>{&g_null};

Stream* S(hipStream_t s) { return s ? reinterpret_cast<Stream*>(s) : &g_null; }

void report(const char* what) {
  ++g_errors;
  fprintf(stderr, "host emulation: %s\n", what);
}

void perform(Op& o) {
  if (o.kind == 1) {
    memset(o.dst, o.value, o.n);
    return;
  }
  if (o.dir == hipMemcpyDeviceToHost) __asan_unpoison_memory_region(o.dst, o.n);
  if (o.dir == hipMemcpyHostToDevice && !o.snap.empty() &&
      memcmp(o.snap.data(), o.src, o.n) != 0)
    report("host source of an asynchronous copy changed before the copy ran");
  memcpy(o.dst, o.src, o.n);
}

void flush(Stream* s, long long upto);

void flush_deps(Stream* s, long long upto) {
  // what this stream waited on before position `upto` must run first
  std::vector<Stream::Dep> d, keep;
  for (const Stream::Dep& p : s->deps) (p.at <= upto ? d : keep).push_back(p);
  s->deps.swap(keep);
  for (const Stream::Dep& p : d)
    if (p.on != s) flush(p.on, p.upto);
}

void flush(Stream* s, long long upto) {
  flush_deps(s, upto);
  size_t k = 0;
  for (; k < s->q.size() && s->q[k].seq <= upto; ++k) perform(s->q[k]);
  s->q.erase(s->q.begin(), s->q.begin() + k);
}

void enqueue(Stream* s, Op o) {
  o.seq = ++g_seq;
  s->last_op_seq = o.seq;
  if (s->capturing) {
    s->graph->nodes.push_back(o);
    return;
  }
  if (o.kind == 0 && o.dir == hipMemcpyHostToDevice)
    o.snap.assign((const char*)o.src, (const char*)o.src + o.n);
  if (o.kind == 0 && o.dir == hipMemcpyDeviceToHost) __asan_poison_memory_region(o.dst, o.n);
  s->q.push_back(std::move(o));
}

bool sync_ok(Stream* s, const char* what) {
  if (s->capturing) {
    report(what);
    return false;
  }
  return true;
}

dim3 g_grid, g_block;
size_t g_shm;
hipStream_t g_stream;

}  // namespace

extern "C" {

long g_launches = 0;
long g_captured_launches = 0;
long emu_errors(void) { return g_errors; }
void emu_flush_all(void) {
  for (Stream* st : g_streams) flush(st, g_seq);
}

void** __hipRegisterFatBinary(const void*) { static void* h[4]; return h; }
void __hipUnregisterFatBinary(void**) {}
void __hipRegisterVar(void**, void*, char*, const char*, int, size_t, int, int) {}
void __hipRegisterFunction(void**, const void*, char*, const char*, unsigned int, void*, void*,
                           dim3*, dim3*, int*) {}
hipError_t __hipPushCallConfiguration(dim3 g, dim3 b, size_t shm, hipStream_t s) {
  g_grid = g; g_block = b; g_shm = shm; g_stream = s; return hipSuccess;
}
hipError_t __hipPopCallConfiguration(dim3* g, dim3* b, size_t* shm, hipStream_t* s) {
  *g = g_grid; *b = g_block; *shm = g_shm; *s = g_stream; return hipSuccess;
}
hipError_t hipLaunchKernel(const void*, dim3 g, dim3 b, void** args, size_t shm, hipStream_t s) {
  ++g_launches;
  // gfx950: 160 KiB of LDS per CU, all of it available to one workgroup
  if (g.x == 0 || g.y == 0 || g.z == 0 || g.y > 65535 || g.z > 65535 || shm > 160 * 1024 ||
      b.x * b.y * b.z > 1024 || !args) {
    fprintf(stderr, "bad launch grid %u %u %u block %u shm %zu\n", g.x, g.y, g.z, b.x, shm);
    abort();
  }
  Stream* st = S(s);
  st->last_op_seq = ++g_seq;
  if (st->capturing) {
    ++g_captured_launches;
    ++st->graph->launches;
  }
  return hipSuccess;
}
hipError_t hipFuncSetAttribute(const void* f, hipFuncAttribute a, int v) {
  if (!f || a != hipFuncAttributeMaxDynamicSharedMemorySize || v < 0 || v > 160 * 1024) {
    fprintf(stderr, "bad function attribute %d = %d\n", (int)a, v);
    abort();
  }
  return hipSuccess;
}
hipError_t hipRuntimeGetVersion(int* v) { *v = HIP_VERSION; return hipSuccess; }
hipError_t hipGetDevice(int* d) { *d = 0; return hipSuccess; }
// a device variable's address is its host shadow (device memory is host memory)
hipError_t hipGetSymbolAddress(void** p, const void* sym) { *p = const_cast<void*>(sym); return hipSuccess; }
hipError_t hipEventCreate(hipEvent_t* e) { *e = (hipEvent_t) new Event(); return hipSuccess; }
hipError_t hipEventCreateWithFlags(hipEvent_t* e, unsigned) { *e = (hipEvent_t) new Event(); return hipSuccess; }
hipError_t hipEventDestroy(hipEvent_t e) { delete (Event*)e; return hipSuccess; }
hipError_t hipEventElapsedTime(float* ms, hipEvent_t, hipEvent_t) { *ms = 1.f; return hipSuccess; }
hipError_t hipEventRecord(hipEvent_t e, hipStream_t s) {
  Event* ev = (Event*)e;
  ev->s = S(s);
  ev->seq = ++g_seq;
  return hipSuccess;
}
hipError_t hipEventSynchronize(hipEvent_t e) {
  Event* ev = (Event*)e;
  if (!ev->s) return hipSuccess;
  if (!sync_ok(ev->s, "event synchronize on a capturing stream")) return hipErrorStreamCaptureUnsupported;
  flush(ev->s, ev->seq);
  return hipSuccess;
}
hipError_t hipStreamWaitEvent(hipStream_t s, hipEvent_t e, unsigned) {
  Event* ev = (Event*)e;
  Stream* st = S(s);
  if (!ev->s) return hipSuccess;
  if (ev->s->capturing && !st->capturing) {
    // fork: this stream joins the capture of the event's stream
    st->capturing = true;
    st->graph = ev->s->graph;
    st->graph->members.insert(st);
    st->last_join_seq = -1;
    st->last_op_seq = ++g_seq;
  }
  if (ev->s->capturing && st->capturing && ev->s != st) ev->s->last_join_seq = ev->seq;
  st->deps.push_back({ev->s, ev->seq, ++g_seq});
  return hipSuccess;
}
const char* hipGetErrorString(hipError_t) { return "emulated error"; }
hipError_t hipGetLastError(void) { return hipSuccess; }
hipError_t hipGraphDestroy(hipGraph_t g) { delete (Graph*)g; return hipSuccess; }
hipError_t hipGraphExecDestroy(hipGraphExec_t g) { delete (Graph*)g; return hipSuccess; }
hipError_t hipGraphInstantiate(hipGraphExec_t* e, hipGraph_t g, hipGraphNode_t*, char*, size_t) {
  *e = (hipGraphExec_t) new Graph(*(Graph*)g);
  return hipSuccess;
}
hipError_t hipGraphLaunch(hipGraphExec_t e, hipStream_t s) {
  Graph* g = (Graph*)e;
  Stream* st = S(s);
  if (st->capturing) {
    report("graph launched on a capturing stream");
    return hipErrorStreamCaptureUnsupported;
  }
  for (const Op& n : g->nodes) enqueue(st, n);
  return hipSuccess;
}
hipError_t hipMemcpyAsync(void* d, const void* s, size_t n, hipMemcpyKind k, hipStream_t st) {
  if (n == 0) return hipSuccess;
  Op o{};
  o.kind = 0; o.dst = d; o.src = s; o.n = n; o.dir = k;
  enqueue(S(st), std::move(o));
  return hipSuccess;
}
hipError_t hipMemsetAsync(void* d, int v, size_t n, hipStream_t st) {
  if (n == 0) return hipSuccess;
  Op o{};
  o.kind = 1; o.dst = d; o.n = n; o.value = v;
  enqueue(S(st), std::move(o));
  return hipSuccess;
}
hipError_t hipStreamBeginCapture(hipStream_t s, hipStreamCaptureMode) {
  Stream* st = S(s);
  if (st->capturing) return hipErrorIllegalState;
  Graph* g = new Graph();
  g->origin = st;
  g->members.insert(st);
  st->capturing = true;
  st->graph = g;
  return hipSuccess;
}
hipError_t hipStreamEndCapture(hipStream_t s, hipGraph_t* out) {
  Stream* st = S(s);
  if (!st->capturing || st->graph->origin != st) return hipErrorIllegalState;
  Graph* g = st->graph;
  hipError_t r = hipSuccess;
  for (Stream* m : g->members) {
    if (m != st && m->last_op_seq > m->last_join_seq) {
      report("capture ended with a forked stream not joined back");
      r = hipErrorStreamCaptureUnjoined;
    }
    m->capturing = false;
    m->graph = nullptr;
    m->deps.clear();
  }
  *out = (hipGraph_t)g;
  return r;
}
hipError_t hipStreamCreateWithFlags(hipStream_t* s, unsigned) {
  Stream* st = new Stream();
  g_streams.push_back(st);
  *s = (hipStream_t)st;
  return hipSuccess;
}
hipError_t hipStreamDestroy(hipStream_t s) {
  Stream* st = S(s);
  if (st->capturing) report("stream destroyed while capturing");
  flush(st, g_seq);  // the runtime completes pending work first
  return hipSuccess;
}
hipError_t hipStreamSynchronize(hipStream_t s) {
  Stream* st = S(s);
  if (!sync_ok(st, "stream synchronize on a capturing stream")) return hipErrorStreamCaptureUnsupported;
  flush(st, g_seq);
  return hipSuccess;
}
hipError_t hipDeviceSynchronize(void) {
  for (Stream* st : g_streams) flush(st, g_seq);
  return hipSuccess;
}
}
