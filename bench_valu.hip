// Issue-rate probe for the VALU instruction classes of the diagonal sweep.
//
// The sweep's VALU roofline counts its algorithmic operations (2 FMA for
// the cross product, MUL + FMA for the key, a row and a column minimum: 6
// per cell) against 64 lanes per CU per clock.  Its compiled loop issues
// other instructions too (key codes, 3-input minima, DPP register shifts,
// lane writes), and the counters show more VALU instructions per CU-clock
// than one.  This program measures, on the device, the sustained issue rate
// of each class alone and of the sweep's per-cell mixes, so that the
// ceiling the sweep is compared with is one the hardware demonstrably
// reaches for that mix.
//
// Each kernel runs `iters` iterations of a fully unrolled body of
// independent register chains (no memory traffic), 256-thread workgroups,
// 8 per CU (8 waves per SIMD); the FP32 mix runs a second time at 4 per CU,
// the occupancy of the FP32 sweep.  Three ways of writing one lane of a
// register other than v_writelane_b32 (a move from a scalar register, a
// select against a lane mask, a move under a one-lane exec mask that the
// same asm statement saves and restores) are timed beside it.  Timing: HIP events around each launch; the shader clock during
// the launch is taken from the core-clock counter (clock64) against the
// constant-rate wall clock (wall_clock64) over the same interval.
// Output: one JSON object on stdout.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstdlib>
#include <vector>

namespace {

enum Kind {
  kFmacF32, kMulF32, kFmaF32, kAndOr, kMin3I32, kMinI32, kDpp, kWritelane,
  kFmaF64, kMulF64, kMinF64, kMixF32, kMixF64,
  kAddF32, kMinF32, kMin3F32, kDppAddF32, kAddU32, kOrB32, kMovS, kCndmask, kMovExec, kCount
};
const char *kName[kCount] = {"v_fmac_f32", "v_mul_f32", "v_fma_f32", "v_and_or_b32", "v_min3_i32",
                             "v_min_i32", "v_mov_b32_dpp", "v_writelane_b32", "v_fma_f64", "v_mul_f64",
                             "v_min_f64", "fp32_sweep_mix", "fp64_sweep_mix", "v_add_f32", "v_min_f32",
                             "v_min3_f32", "v_add_f32_dpp", "v_add_u32", "v_or_b32", "v_mov_b32_from_sgpr",
                             "v_cndmask_b32_lane_mask", "v_mov_b32_exec_one_lane"};

// Instructions per unrolled body, per kind.
constexpr int kBodyFp32Mix = 48 + 24 + 24 + 24 + 21 + 4 + 8 + 8;   // 161 for 24 cells
constexpr int kBodyFp64Mix = 16 + 8 + 8 + 8 + 16 + 10 + 8;         // 74 for 8 cells
int body_len(int k) {
  if (k == kMixF32) return kBodyFp32Mix;
  if (k == kMixF64) return kBodyFp64Mix;
  return 16;
}

#define FMAC(r) asm volatile("v_fmac_f32 %0, %1, %2" : "+v"(f[r]) : "v"(x), "v"(y))
#define MULF(r) asm volatile("v_mul_f32 %0, %0, %1" : "+v"(f[r]) : "v"(y))
#define FMAF(r) asm volatile("v_fma_f32 %0, %1, %2, %0" : "+v"(f[r]) : "v"(x), "v"(y))
#define FMAG(r) asm volatile("v_fma_f32 %0, %1, %2, %0" : "+v"(g[r]) : "v"(x), "v"(y))
#define MULG(r) asm volatile("v_mul_f32 %0, %0, %1" : "+v"(g[r]) : "v"(y))
#define MIN3V(r) asm volatile("v_min3_i32 %0, %0, %1, %2" : "+v"(v[r]) : "v"(p), "v"(q))
#define MINV(r) asm volatile("v_min_i32 %0, %0, %1" : "+v"(v[r]) : "v"(p))
#define ANDOR(r) asm volatile("v_and_or_b32 %0, %0, %1, %2" : "+v"(u[r]) : "v"(mask), "v"(code))
#define MIN3(r) asm volatile("v_min3_i32 %0, %0, %1, %2" : "+v"(u[r]) : "v"(p), "v"(q))
#define MINI(r) asm volatile("v_min_i32 %0, %0, %1" : "+v"(u[r]) : "v"(p))
#define DPP(r) asm volatile("v_mov_b32_dpp %0, %1 wave_shl:1 row_mask:0xf bank_mask:0xf" : "=v"(w[r]) : "v"(w[(r) + 1]))
#define WLANE(r) asm volatile("v_writelane_b32 %0, %1, 63" : "+v"(w[r]) : "s"(fill))
#define FMAD(r) asm volatile("v_fma_f64 %0, %1, %2, %0" : "+v"(d[r]) : "v"(dx), "v"(dy))
#define MULD(r) asm volatile("v_mul_f64 %0, %0, %1" : "+v"(d[r]) : "v"(dy))
#define MIND(r) asm volatile("v_min_f64 %0, %0, %1" : "+v"(e[r]) : "v"(dy))
#define ADDF(r) asm volatile("v_add_f32 %0, %0, %1" : "+v"(f[r]) : "v"(y))
#define MINF(r) asm volatile("v_min_f32 %0, %0, %1" : "+v"(f[r]) : "v"(y))
#define MIN3F(r) asm volatile("v_min3_f32 %0, %0, %1, %2" : "+v"(f[r]) : "v"(x), "v"(y))
#define DPPADD(r) asm volatile("v_add_f32_dpp %0, %1, %2 wave_shl:1 row_mask:0xf bank_mask:0xf" : "=v"(g[r]) : "v"(g[((r) + 1) & 15]), "v"(y))
#define ADDU(r) asm volatile("v_add_u32 %0, %0, %1" : "+v"(u[r]) : "v"(p))
#define ORB(r) asm volatile("v_or_b32 %0, %0, %1" : "+v"(u[r]) : "v"(p))
#define MOVS(r) asm volatile("v_mov_b32 %0, %1" : "=v"(w[r]) : "s"(fill))
#define CNDM(r) asm volatile("v_cndmask_b32_e64 %0, %0, %1, %2" : "+v"(w[r]) : "v"(fillv), "s"(m63))
#define MOVX(r) asm volatile("s_mov_b64 %1, exec\n s_mov_b64 exec, %2\n v_mov_b32 %0, %3\n s_mov_b64 exec, %1" : "+v"(w[r]), "=&s"(sv) : "s"(m63), "s"(fill))
#define MOVB(r) asm volatile("v_mov_b32 %0, %1" : "=v"(w[r]) : "v"(w[(r) - 8]))

#define R16(M) M(0); M(1); M(2); M(3); M(4); M(5); M(6); M(7); M(8); M(9); M(10); M(11); M(12); M(13); M(14); M(15)
#define R8(M) M(0); M(1); M(2); M(3); M(4); M(5); M(6); M(7)
#define R8B(M) M(8); M(9); M(10); M(11); M(12); M(13); M(14); M(15)

template <int K>
__global__ void __launch_bounds__(256) k_probe(float *out, unsigned long long *clk, int iters, float seed, int fill) {
  float f[16], g[16];
  int u[16], v[16];
  int w[17];
  double d[16], e[16];
  for (int r = 0; r < 16; ++r) {
    f[r] = seed + (float)(threadIdx.x + r);
    g[r] = seed - (float)r;
    u[r] = (int)threadIdx.x * 16 + r;
    v[r] = (int)threadIdx.x - r;
    w[r] = r * 3 + (int)threadIdx.x;
    d[r] = (double)f[r];
    e[r] = (double)u[r];
  }
  w[16] = (int)threadIdx.x;
  const float x = seed * 0.5f, y = 1.0f - seed * 1e-3f;
  const int mask = ~1023, code = (int)(threadIdx.x & 1023), p = (int)threadIdx.x, q = 7;
  const double dx = (double)x, dy = (double)y;
  const unsigned long long m63 = 1ull << 63;  // lane 63
  const int fillv = (int)threadIdx.x + fill;
  unsigned long long sv;
  const unsigned long long c0 = clock64(), t0 = wall_clock64();
  for (int it = 0; it < iters; ++it) {
    if constexpr (K == kFmacF32) { R16(FMAC); }
    if constexpr (K == kMulF32) { R16(MULF); }
    if constexpr (K == kFmaF32) { R16(FMAF); }
    if constexpr (K == kAndOr) { R16(ANDOR); }
    if constexpr (K == kMin3I32) { R16(MIN3); }
    if constexpr (K == kMinI32) { R16(MINI); }
    if constexpr (K == kDpp) { R16(DPP); }
    if constexpr (K == kWritelane) { R16(WLANE); }
    if constexpr (K == kFmaF64) { R16(FMAD); }
    if constexpr (K == kMulF64) { R16(MULD); }
    if constexpr (K == kMinF64) { R16(MIND); }
    if constexpr (K == kAddF32) { R16(ADDF); }
    if constexpr (K == kMinF32) { R16(MINF); }
    if constexpr (K == kMin3F32) { R16(MIN3F); }
    if constexpr (K == kDppAddF32) { R16(DPPADD); }
    if constexpr (K == kAddU32) { R16(ADDU); }
    if constexpr (K == kOrB32) { R16(ORB); }
    if constexpr (K == kMovS) { R16(MOVS); }
    if constexpr (K == kCndmask) { R16(CNDM); }
    if constexpr (K == kMovExec) { R16(MOVX); }
    if constexpr (K == kMixF32) {
      // 24 cells of the FP32 sweep's loop: 48 v_fmac + 24 v_fma + 24 v_mul
      // (cross products and keys), 24 v_and_or (codes), 21 v_min3 + 4 v_min
      // (row and column minima), 8 DPP shifts + 8 lane writes (rotation),
      // interleaved so that no instruction waits on the one before it
      DPP(0); FMAC(0); FMAC(1); FMAC(2); FMAG(0); FMAC(3); FMAC(4); FMAC(5); WLANE(0); FMAG(1); ANDOR(0); FMAG(2); MULG(8); MULG(9); MULG(10); ANDOR(1); ANDOR(2); MIN3V(0); MIN3V(1); MIN3V(2); MINV(11);
      DPP(1); FMAC(6); FMAC(7); FMAC(8); FMAG(6); FMAC(9); FMAC(10); FMAC(11); WLANE(1); FMAG(7); ANDOR(3); FMAG(8); MULG(14); MULG(15); MULG(0); ANDOR(4); ANDOR(5); MIN3V(3); MIN3V(4); MIN3V(5); MINV(14);
      DPP(2); FMAC(12); FMAC(13); FMAC(14); FMAG(12); FMAC(15); FMAC(0); FMAC(1); WLANE(2); FMAG(13); ANDOR(6); FMAG(14); MULG(4); MULG(5); MULG(6); ANDOR(7); ANDOR(8); MIN3V(6); MIN3V(7); MIN3V(8); MINV(1);
      DPP(3); FMAC(2); FMAC(3); FMAC(4); FMAG(2); FMAC(5); FMAC(6); FMAC(7); WLANE(3); FMAG(3); ANDOR(9); FMAG(4); MULG(10); MULG(11); MULG(12); ANDOR(10); ANDOR(11); MIN3V(9); MIN3V(10); MIN3V(11); MINV(4);
      DPP(4); FMAC(8); FMAC(9); FMAC(10); FMAG(8); FMAC(11); FMAC(12); FMAC(13); WLANE(4); FMAG(9); ANDOR(12); FMAG(10); MULG(0); MULG(1); MULG(2); ANDOR(13); ANDOR(14); MIN3V(12); MIN3V(13); MIN3V(14);
      DPP(5); FMAC(14); FMAC(15); FMAC(0); FMAG(14); FMAC(1); FMAC(2); FMAC(3); WLANE(5); FMAG(15); ANDOR(15); FMAG(0); MULG(6); MULG(7); MULG(8); ANDOR(0); ANDOR(1); MIN3V(15); MIN3V(0);
      DPP(6); FMAC(4); FMAC(5); FMAC(6); FMAG(4); FMAC(7); FMAC(8); FMAC(9); WLANE(6); FMAG(5); ANDOR(2); FMAG(6); MULG(12); MULG(13); MULG(14); ANDOR(3); ANDOR(4); MIN3V(1); MIN3V(2);
      DPP(7); FMAC(10); FMAC(11); FMAC(12); FMAG(10); FMAC(13); FMAC(14); FMAC(15); WLANE(7); FMAG(11); ANDOR(5); FMAG(12); MULG(2); MULG(3); MULG(4); ANDOR(6); ANDOR(7); MIN3V(3); MIN3V(4);
    }
    if constexpr (K == kMixF64) {
      // 8 cells of the FP64 sweep's loop: 16 v_fma_f64 (cross products; the
      // compiler's v_fmac_f64 is the same operation) + 8 v_fma_f64 + 8
      // v_mul_f64 (keys), 8 v_and_or (codes), 16 v_min_f64 (row and column
      // minima), 10 DPP moves (rotation of four FP64 records + lane-pair
      // exchange) and 8 register moves
      DPP(0); FMAD(0); FMAD(1); FMAD(2); MOVB(8); MULD(8); ANDOR(0); MIND(0); MIND(1);
      DPP(1); FMAD(3); FMAD(4); FMAD(5); MOVB(9); MULD(11); ANDOR(1); MIND(2); MIND(3);
      DPP(2); FMAD(6); FMAD(7); FMAD(8); MOVB(10); MULD(14); ANDOR(2); MIND(4); MIND(5); DPP(8);
      DPP(3); FMAD(9); FMAD(10); FMAD(11); MOVB(11); MULD(1); ANDOR(3); MIND(6); MIND(7);
      DPP(4); FMAD(12); FMAD(13); FMAD(14); MOVB(12); MULD(4); ANDOR(4); MIND(8); MIND(9);
      DPP(5); FMAD(15); FMAD(0); FMAD(1); MOVB(13); MULD(7); ANDOR(5); MIND(10); MIND(11); DPP(9);
      DPP(6); FMAD(2); FMAD(3); FMAD(4); MOVB(14); MULD(10); ANDOR(6); MIND(12); MIND(13);
      DPP(7); FMAD(5); FMAD(6); FMAD(7); MOVB(15); MULD(13); ANDOR(7); MIND(14); MIND(15);
    }
  }
  const unsigned long long c1 = clock64(), t1 = wall_clock64();
  float acc = 0.f;
  for (int r = 0; r < 16; ++r) acc += f[r] + g[r] + (float)u[r] + (float)v[r] + (float)w[r] + (float)d[r] + (float)e[r];
  out[blockIdx.x * blockDim.x + threadIdx.x] = acc;
  if (threadIdx.x == 0) {
    clk[2 * blockIdx.x] = c1 - c0;
    clk[2 * blockIdx.x + 1] = t1 - t0;
  }
}

template <int K>
void run(int cus, int iters, int blocks_per_cu, float *out, unsigned long long *clk, double wall_mhz, FILE *js,
         bool last, const char *label = nullptr) {
  const int grid = cus * blocks_per_cu;
  hipEvent_t a, b;
  (void)hipEventCreate(&a);
  (void)hipEventCreate(&b);
  hipLaunchKernelGGL(k_probe<K>, dim3(grid), dim3(256), 0, 0, out, clk, iters / 8, 1.0f, 3);  // warm-up
  (void)hipEventRecord(a, 0);
  hipLaunchKernelGGL(k_probe<K>, dim3(grid), dim3(256), 0, 0, out, clk, iters, 1.0f, 3);
  (void)hipEventRecord(b, 0);
  (void)hipEventSynchronize(b);
  float ms = 0.f;
  (void)hipEventElapsedTime(&ms, a, b);
  std::vector<unsigned long long> h(2 * (size_t)grid);
  (void)hipMemcpy(h.data(), clk, h.size() * 8, hipMemcpyDeviceToHost);
  double cyc = 0, wall = 0;
  for (int i = 0; i < grid; ++i) {
    cyc += (double)h[2 * i];
    wall += (double)h[2 * i + 1];
  }
  const double mhz = wall > 0 ? cyc / wall * wall_mhz : 0.0;  // core clock during the loop
  const int body = body_len(K);
  const double waves = (double)grid * 4.0;
  const double winst = waves * (double)iters * body;
  const double secs = ms * 1e-3;
  const double per_cu_clk = winst / (secs * cus * mhz * 1e6);
  const double lane_rate = winst * 64.0 / secs;
  std::fprintf(js, "  \"%s\": {\"ms\": %.4f, \"wave_instructions\": %.6e, \"lane_instructions_per_s\": %.6e, "
                   "\"core_clock_mhz\": %.1f, \"wave_instructions_per_cu_clock\": %.4f}%s\n",
               label ? label : kName[K], ms, winst, lane_rate, mhz, per_cu_clk, last ? "" : ",");
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
}

}  // namespace

int main(int argc, char **argv) {
  const int iters = argc > 1 ? std::atoi(argv[1]) : 20000;
  int dev = 0, cus = 0, wall_khz = 0;
  if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) {
    std::fprintf(stderr, "no device\n");
    return 1;
  }
  if (hipDeviceGetAttribute(&wall_khz, hipDeviceAttributeWallClockRate, dev) != hipSuccess || wall_khz <= 0) wall_khz = 100000;
  const int bpc = 8;
  float *out = nullptr;
  unsigned long long *clk = nullptr;
  if (hipMalloc(&out, sizeof(float) * 256 * cus * bpc) != hipSuccess ||
      hipMalloc(&clk, sizeof(unsigned long long) * 2 * cus * bpc) != hipSuccess) {
    std::fprintf(stderr, "allocation failed\n");
    return 1;
  }
  const double wall_mhz = wall_khz / 1000.0;
  std::printf("{\"cus\": %d, \"wall_clock_mhz\": %.1f, \"iters\": %d, \"workgroups_per_cu\": %d,\n", cus, wall_mhz,
              iters, bpc);
  FILE *js = stdout;
  run<kFmacF32>(cus, iters, bpc, out, clk, wall_mhz, js, false);
  run<kMulF32>(cus, iters, bpc, out, clk, wall_mhz, js, false);
  run<kFmaF32>(cus, iters, bpc, out, clk, wall_mhz, js, false);
  run<kAndOr>(cus, iters, bpc, out, clk, wall_mhz, js, false);
  run<kMin3I32>(cus, iters, bpc, out, clk, wall_mhz, js, false);
  run<kMinI32>(cus, iters, bpc, out, clk, wall_mhz, js, false);
  run<kDpp>(cus, iters, bpc, out, clk, wall_mhz, js, false);
  run<kWritelane>(cus, iters, bpc, out, clk, wall_mhz, js, false);
  run<kFmaF64>(cus, iters, bpc, out, clk, wall_mhz, js, false);
  run<kMulF64>(cus, iters, bpc, out, clk, wall_mhz, js, false);
  run<kMinF64>(cus, iters, bpc, out, clk, wall_mhz, js, false);
  run<kMixF32>(cus, iters / 8, bpc, out, clk, wall_mhz, js, false);
  run<kMixF64>(cus, iters / 4, bpc, out, clk, wall_mhz, js, false);
  run<kAddF32>(cus, iters, bpc, out, clk, wall_mhz, js, false);
  run<kMinF32>(cus, iters, bpc, out, clk, wall_mhz, js, false);
  run<kMin3F32>(cus, iters, bpc, out, clk, wall_mhz, js, false);
  run<kDppAddF32>(cus, iters, bpc, out, clk, wall_mhz, js, false);
  run<kAddU32>(cus, iters, bpc, out, clk, wall_mhz, js, false);
  run<kOrB32>(cus, iters, bpc, out, clk, wall_mhz, js, false);
  run<kMovS>(cus, iters, bpc, out, clk, wall_mhz, js, false);
  run<kCndmask>(cus, iters, bpc, out, clk, wall_mhz, js, false);
  run<kMovExec>(cus, iters, bpc, out, clk, wall_mhz, js, false);
  run<kMixF32>(cus, iters / 8, 4, out, clk, wall_mhz, js, true, "fp32_sweep_mix_4_waves_per_simd");
  std::printf("}\n");
  (void)hipFree(out);
  (void)hipFree(clk);
  return 0;
}
