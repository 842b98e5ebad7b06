// Scheduler of the CPU stand-in for the HIP runtime (tests only): the threads
// of a block are fibers that run until they reach a barrier or a wavefront
// collective; a barrier opens once every live thread of the block (or of the
// wavefront) has reached it.  A collective reached by only part of a
// wavefront, or a block waiting on two different barriers, is reported and
// aborts the run.  A thread that sleeps or fences (as the persistent kernel
// does while it waits and between its work items) parks its block: the
// scheduler goes on with another block (starting the next one while fewer
// than SLOTS are under way) and comes back to the parked one in turn, so
// blocks that wait on each other's progress interleave.  A block runs alone
// between its parking points (LDS, static here, is shared by the blocks
// under way).
#include <time.h>
#include <hip/hip_runtime.h>

#include <vector>

#if defined(__has_feature)
#if __has_feature(address_sanitizer)
#define EMU_ASAN 1
#endif
#endif
#ifdef EMU_ASAN
#include <sanitizer/common_interface_defs.h>
#endif

// Context switch (x86-64 System V): saves the callee-saved registers on the
// current stack, stores the stack pointer to *save, loads `load` and
// restores the registers saved there (ucontext's switches make a system call
// each).
extern "C" void emu_switch(void **save, void *load);
asm(R"(
  .text
  .globl emu_switch
  .type emu_switch,@function
emu_switch:
  pushq %rbp
  pushq %rbx
  pushq %r12
  pushq %r13
  pushq %r14
  pushq %r15
  movq %rsp, (%rdi)
  movq %rsi, %rsp
  popq %r15
  popq %r14
  popq %r13
  popq %r12
  popq %rbx
  popq %rbp
  ret
  .size emu_switch, .-emu_switch
)");

namespace emu {

enum { RUN = 0, AT_BARRIER = 1, AT_WAVE = 2, DONE = 3, PARKED = 4 };

struct Fiber {
  void *sp = nullptr;  // saved stack pointer while switched out
  char *stack = nullptr;
  size_t ssize = 0;
  dim3 tid;
  int lane = 0, wave = 0;
  int state = RUN;
  unsigned wgen = 0;  // wavefront collectives passed
  void *fake = nullptr;
};

struct Wave {
  uint64_t buf[2][64];
};

// A block under way: its threads are fibers[f0, f0 + nt) of the pool.
struct Block {
  uint32_t idx = 0;
  int f0 = 0;
  std::vector<Wave> waves;
};
static const int SLOTS = 8;

Fiber *cur = nullptr;
dim3 block_idx, grid_dim, block_dim;
static void *sched_sp = nullptr;
static const void *sched_bottom = nullptr;
static size_t sched_size = 0;
static std::vector<Fiber> fibers;
static Block *cur_block = nullptr;
static int cur_nt = 0;
static const std::function<void()> *body = nullptr;
static const size_t STACK = 1 << 20;
void (*after_launch)() = nullptr;  // set by a test driver: checks after every launch

const dim3 &thread_idx() { return cur->tid; }
int lane_id() { return cur->lane; }

static void die(const char *what) {
  fprintf(stderr, "emu: %s (block %u, thread %u)\n", what, block_idx.x, cur ? cur->tid.x : 0u);
  abort();
}

static void yield_to_scheduler() {
#ifdef EMU_ASAN
  void *fake = nullptr;
  __sanitizer_start_switch_fiber(&fake, sched_bottom, sched_size);
  emu_switch(&cur->sp, sched_sp);
  __sanitizer_finish_switch_fiber(fake, &sched_bottom, &sched_size);
#else
  emu_switch(&cur->sp, sched_sp);
#endif
}

static void entry() {
#ifdef EMU_ASAN
  __sanitizer_finish_switch_fiber(nullptr, &sched_bottom, &sched_size);
#endif
  (*body)();
  cur->state = DONE;
#ifdef EMU_ASAN
  __sanitizer_start_switch_fiber(nullptr, sched_bottom, sched_size);
#endif
  void *dead;
  emu_switch(&dead, sched_sp);  // never resumed
  abort();
}

// A fresh stack whose first switch-in "returns" into entry() with the
// alignment of a call (rsp = 8 mod 16 on entry).
static void *fresh_stack(Fiber &f) {
  uintptr_t top = ((uintptr_t)f.stack + f.ssize) & ~(uintptr_t)15;
  void **sp = (void **)top;
  *--sp = nullptr;          // entry()'s return address: never used
  *--sp = (void *)&entry;   // emu_switch returns here
  for (int r = 0; r < 6; r++) *--sp = nullptr;  // rbp rbx r12 r13 r14 r15
  return (void *)sp;
}

void block_barrier() {
  cur->state = AT_BARRIER;
  yield_to_scheduler();
}

long parks = 0;         // sleeps and fences that parked a thread (read by test drivers)
long blocks_waited = 0;  // times the scheduler turned to another block

void sleep_park() {
  parks++;
  cur->state = PARKED;
  yield_to_scheduler();
}

const uint64_t *wave_exchange(uint64_t v) {
  const unsigned g = cur->wgen++ & 1u;
  std::vector<Wave> &waves = cur_block->waves;
  waves[cur->wave].buf[g][cur->lane] = v;
  cur->state = AT_WAVE;
  yield_to_scheduler();
  return waves[cur->wave].buf[g];
}

static void run_fiber(Fiber &f) {
  cur = &f;
#ifdef EMU_ASAN
  void *fake = nullptr;
  __sanitizer_start_switch_fiber(&fake, f.stack, f.ssize);
  emu_switch(&sched_sp, f.sp);
  __sanitizer_finish_switch_fiber(fake, nullptr, nullptr);
#else
  emu_switch(&sched_sp, f.sp);
#endif
  cur = nullptr;
}

// Opens the barriers of block B whose threads have all arrived; false when
// none could.
static bool release(Block &B) {
  bool any = false;
  const int nt = cur_nt;
  Fiber *fib = &fibers[B.f0];
  std::vector<Wave> &waves = B.waves;
  for (size_t w = 0; w < waves.size(); w++) {
    int waiting = 0, live = 0;
    unsigned gen = 0;
    bool mixed = false;
    for (int t = (int)w * 64; t < nt && t < (int)(w + 1) * 64; t++) {
      Fiber &f = fib[t];
      if (f.state == DONE) continue;
      live++;
      if (f.state == AT_WAVE) {
        if (waiting && f.wgen != gen) mixed = true;
        gen = f.wgen;
        waiting++;
      }
    }
    if (!waiting || waiting != live) continue;
    if (mixed) die("lanes of one wavefront at different collectives");
    const unsigned g = (gen - 1) & 1u;  // the buffer of the collective they wait at
    for (int l = 0; l < 64; l++) {
      const int t = (int)w * 64 + l;
      if (t >= nt || fib[t].state == DONE) waves[w].buf[g][l] = 0;
    }
    for (int t = (int)w * 64; t < nt && t < (int)(w + 1) * 64; t++)
      if (fib[t].state == AT_WAVE) fib[t].state = RUN;
    any = true;
  }
  if (any) return true;
  int live = 0, bar = 0;
  for (int t = 0; t < nt; t++) {
    if (fib[t].state == DONE) continue;
    live++;
    bar += fib[t].state == AT_BARRIER;
  }
  if (live && bar == live) {
    for (int t = 0; t < nt; t++)
      if (fib[t].state == AT_BARRIER) fib[t].state = RUN;
    return true;
  }
  return false;
}

// Runs block B until it finishes (true) or one of its threads parks (false).
static bool run_block(Block &B) {
  block_idx = dim3(B.idx);
  cur_block = &B;
  Fiber *fib = &fibers[B.f0];
  for (int t = 0; t < cur_nt; t++)
    if (fib[t].state == PARKED) fib[t].state = RUN;
  for (;;) {
    bool ran = false, parked = false;
    for (int t = 0; t < cur_nt; t++)
      if (fib[t].state == RUN) {
        run_fiber(fib[t]);
        ran = true;
        parked |= fib[t].state == PARKED;
      }
    int done = 0;
    for (int t = 0; t < cur_nt; t++) done += fib[t].state == DONE;
    if (done == cur_nt) return true;
    if (parked) return false;
    if (ran) continue;
    if (!release(B)) die("deadlock: threads wait at different barriers");
  }
}

void launch(dim3 grid, dim3 block, const std::function<void()> &fn) {
  if (block.y != 1 || block.z != 1 || grid.y != 1 || grid.z != 1) die("only 1-D launches are emulated");
  const int nt = (int)block.x;
  if (nt <= 0 || nt > 1024) die("bad block size");
  const size_t need = (size_t)SLOTS * nt;
  if (fibers.size() < need) {
    size_t old = fibers.size();
    fibers.resize(need);
    for (size_t t = old; t < fibers.size(); t++) {
      fibers[t].stack = (char *)malloc(STACK);
      fibers[t].ssize = STACK;
    }
  }
  grid_dim = grid;
  block_dim = block;
  body = &fn;
  cur_nt = nt;
  std::vector<Block> slot(SLOTS);
  std::vector<int> active;  // slots under way, in turn order
  std::vector<int> free_slots;
  for (int k = SLOTS - 1; k >= 0; k--) free_slots.push_back(k);
  uint32_t next = 0;
  auto start = [&](uint32_t b) {
    const int k = free_slots.back();
    free_slots.pop_back();
    Block &B = slot[k];
    B.idx = b;
    B.f0 = k * nt;
    B.waves.assign((nt + 63) / 64, Wave{});
    for (int t = 0; t < nt; t++) {
      Fiber &f = fibers[B.f0 + t];
      f.tid = dim3((uint32_t)t);
      f.lane = t & 63;
      f.wave = t >> 6;
      f.state = RUN;
      f.wgen = 0;
      f.sp = fresh_stack(f);
    }
    active.push_back(k);
  };
  while (next < grid.x || !active.empty()) {
    if (active.empty()) start(next++);
    const int k = active.front();
    active.erase(active.begin());
    if (run_block(slot[k])) {
      free_slots.push_back(k);
      continue;
    }
    // parked: another block goes first (a new one while a slot is free)
    blocks_waited++;
    if (next < grid.x && !free_slots.empty()) start(next++);
    active.push_back(k);
  }
  cur_block = nullptr;
  body = nullptr;
  if (after_launch) after_launch();
}

}  // namespace emu

// ---- host API -------------------------------------------------------------
struct emu_event_t {
  int unused;
};
struct emu_stream_t {
  int unused;
};

hipError_t hipMalloc(void **p, size_t bytes) {
  *p = malloc(bytes ? bytes : 1);
  return *p ? hipSuccess : hipErrorOutOfMemory;
}
hipError_t hipFree(void *p) {
  free(p);
  return hipSuccess;
}
hipError_t hipMallocAsync(void **p, size_t bytes, hipStream_t) { return hipMalloc(p, bytes); }
hipError_t hipFreeAsync(void *p, hipStream_t) { return hipFree(p); }
hipError_t hipMemcpy(void *d, const void *s, size_t bytes, hipMemcpyKind) {
  if (bytes) memmove(d, s, bytes);
  return hipSuccess;
}
hipError_t hipMemcpyAsync(void *d, const void *s, size_t bytes, hipMemcpyKind k, hipStream_t) {
  return hipMemcpy(d, s, bytes, k);
}
hipError_t hipMemsetAsync(void *d, int v, size_t bytes, hipStream_t) {
  memset(d, v, bytes);
  return hipSuccess;
}
hipError_t hipStreamSynchronize(hipStream_t) { return hipSuccess; }
hipError_t hipDeviceSynchronize() { return hipSuccess; }
hipError_t hipGetLastError() { return hipSuccess; }
hipError_t hipPeekAtLastError() { return hipSuccess; }
const char *hipGetErrorString(hipError_t e) { return e == hipSuccess ? "no error" : "emulated error"; }
hipError_t hipEventCreate(hipEvent_t *e) {
  *e = new emu_event_t();
  return hipSuccess;
}
hipError_t hipEventCreateWithFlags(hipEvent_t *e, unsigned) { return hipEventCreate(e); }
hipError_t hipEventDestroy(hipEvent_t e) {
  delete e;
  return hipSuccess;
}
hipError_t hipEventRecord(hipEvent_t, hipStream_t) { return hipSuccess; }
hipError_t hipEventSynchronize(hipEvent_t) { return hipSuccess; }
hipError_t hipEventElapsedTime(float *ms, hipEvent_t, hipEvent_t) {
  *ms = 1.0f;
  return hipSuccess;
}
hipError_t hipStreamCreateWithFlags(hipStream_t *s, unsigned) {
  *s = new emu_stream_t();
  return hipSuccess;
}
hipError_t hipStreamDestroy(hipStream_t s) {
  delete s;
  return hipSuccess;
}
hipError_t hipStreamWaitEvent(hipStream_t, hipEvent_t, unsigned) { return hipSuccess; }
hipError_t hipStreamBeginCapture(hipStream_t, hipStreamCaptureMode) { return hipErrorNotSupported; }
hipError_t hipStreamEndCapture(hipStream_t, hipGraph_t *) { return hipErrorNotSupported; }
hipError_t hipGraphInstantiate(hipGraphExec_t *, hipGraph_t, hipGraphNode_t *, char *, size_t) {
  return hipErrorNotSupported;
}
hipError_t hipGraphLaunch(hipGraphExec_t, hipStream_t) { return hipErrorNotSupported; }
hipError_t hipGraphExecDestroy(hipGraphExec_t) { return hipSuccess; }
hipError_t hipGraphDestroy(hipGraph_t) { return hipSuccess; }
hipError_t hipLaunchKernel(const void *, dim3, dim3, void **, size_t, hipStream_t) { return hipErrorNotSupported; }
// four "CUs" holding one block each; a wall clock of 100 MHz
hipError_t hipDeviceGetAttribute(int *v, int attr, int) {
  if (attr == hipDeviceAttributeMultiprocessorCount) {
    *v = 4;
    return hipSuccess;
  }
  if (attr == hipDeviceAttributeWallClockRate) {
    *v = 100000;
    return hipSuccess;
  }
  return hipErrorNotSupported;
}
hipError_t hipOccupancyMaxActiveBlocksPerMultiprocessor(int *nb, const void *, int, size_t) {
  *nb = 1;
  return hipSuccess;
}
// ticks at a tenth of the 100 MHz it claims: emulated kernels run far slower
// than the device, and a launch-wide deadline must not pass for that alone
uint64_t wall_clock64() {
  struct timespec t;
  clock_gettime(CLOCK_MONOTONIC, &t);
  return (uint64_t)t.tv_sec * 10000000ull + (uint64_t)t.tv_nsec / 100ull;
}
hipError_t hipGetDevice(int *d) {
  *d = 0;
  return hipSuccess;
}
hipError_t hipGetSymbolAddress(void **p, const void *symbol) {
  *p = (void *)symbol;
  return hipSuccess;
}
