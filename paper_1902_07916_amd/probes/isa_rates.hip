// isa_rates.hip -- throughput probe for the gfx950 instruction classes the
// sampling kernel uses: each thread runs 8 independent chains of one
// instruction (or 8 chains each of two instructions, for the mixes), 4096
// blocks of 256 threads, timed with HIP events.  Prints lanes per clock per
// CU at 256 CUs and 2.4 GHz.  Build:
//   hipcc -O3 --offload-arch=gfx950 -Xclang -target-feature -Xclang -packed-fp32-ops \
//         -I include -I paper_1902_07916_amd/csrc paper_1902_07916_amd/probes/isa_rates.hip -o isa_rates
#include <hip/hip_runtime.h>
#include <cstdio>
#include <cstdint>
#define R 2048
__global__ void k_mad(uint32_t* out, uint32_t s) {
  uint64_t p[8];
  for (int i=0;i<8;i++){p[i]=threadIdx.x*8+i+s+((uint64_t)blockIdx.x<<32);}
  for (int r=0;r<R;r++){
#pragma unroll
    for (int i=0;i<8;i++){ p[i]=(uint64_t)(uint32_t)p[i]*0xD2511F53u + p[i];} }
  uint32_t a=0; for(int i=0;i<8;i++) a^=(uint32_t)p[i]^(uint32_t)(p[i]>>32);
  out[blockIdx.x*blockDim.x+threadIdx.x]=a;
}
#include "zmc_device.hpp"
// 8 Philox blocks per iteration (independent counters), like the sampler
__global__ void k_philox(uint32_t* out, uint32_t s) {
  uint32_t acc = 0;
  const uint32_t base = (blockIdx.x*blockDim.x+threadIdx.x)*8;
  for (int r=0;r<R/8;r++){
#pragma unroll
    for (int i=0;i<8;i++){ zmc::U4 v = zmc::philox4x32_10(base + r*8*1048576u + i, s, 7u, 9u, 11u, s*3u); acc ^= v.x ^ v.y ^ v.z ^ v.w; } }
  out[blockIdx.x*blockDim.x+threadIdx.x]=acc;
}
__global__ void k_bitop3(uint32_t* out, uint32_t s) {
  uint32_t x[8]; for (int i=0;i<8;i++) x[i]=threadIdx.x*8+i+s;
  uint32_t y=blockIdx.x*77+s, z=s*3+1;
  for (int r=0;r<R;r++){
#pragma unroll
    for (int i=0;i<8;i++) x[i]=__builtin_amdgcn_bitop3_b32(x[i], x[(i+1)&7], z+i, 0x96); }
  uint32_t a=0; for(int i=0;i<8;i++) a^=x[i];
  out[blockIdx.x*blockDim.x+threadIdx.x]=a+y;
}
__global__ void k_fma32(float* out, float s) {
  float x[8]; for (int i=0;i<8;i++) x[i]=threadIdx.x*1e-3f+i+s;
  for (int r=0;r<R;r++){
#pragma unroll
    for (int i=0;i<8;i++) x[i]=__builtin_fmaf(x[i], 0.999f, 0.001f); }
  float a=0; for(int i=0;i<8;i++) a+=x[i];
  out[blockIdx.x*blockDim.x+threadIdx.x]=a;
}
__global__ void k_fma64(double* out, double s) {
  double x[8]; for (int i=0;i<8;i++) x[i]=threadIdx.x*1e-3+i+s;
  for (int r=0;r<R;r++){
#pragma unroll
    for (int i=0;i<8;i++) x[i]=fma(x[i], 0.999, 0.001); }
  double a=0; for(int i=0;i<8;i++) a+=x[i];
  out[blockIdx.x*blockDim.x+threadIdx.x]=a;
}
__global__ void k_sin(float* out, float s) {
  float x[8]; for (int i=0;i<8;i++) x[i]=threadIdx.x*1e-3f+i*0.1f+s;
  for (int r=0;r<R;r++){
#pragma unroll
    for (int i=0;i<8;i++) x[i]=__builtin_amdgcn_sinf(x[i]); }
  float a=0; for(int i=0;i<8;i++) a+=x[i];
  out[blockIdx.x*blockDim.x+threadIdx.x]=a;
}
__global__ void k_exp(float* out, float s) {
  float x[8]; for (int i=0;i<8;i++) x[i]=-(threadIdx.x*1e-3f+i*0.1f+s);
  for (int r=0;r<R;r++){
#pragma unroll
    for (int i=0;i<8;i++) x[i]=-__builtin_amdgcn_exp2f(x[i]); }
  float a=0; for(int i=0;i<8;i++) a+=x[i];
  out[blockIdx.x*blockDim.x+threadIdx.x]=a;
}
__global__ void k_add64(double* out, float s) {
  double acc[8]; float x[8];
  for (int i=0;i<8;i++){acc[i]=0; x[i]=threadIdx.x*1e-3f+i+s;}
  for (int r=0;r<R;r++){
#pragma unroll
    for (int i=0;i<8;i++){ acc[i] += (double)x[i]; x[i] = x[i]*1.0001f; } }
  double a=0; for(int i=0;i<8;i++) a+=acc[i];
  out[blockIdx.x*blockDim.x+threadIdx.x]=a;
}
__global__ void k_alignbit(uint32_t* out, uint32_t s) {
  uint32_t x[8]; for (int i=0;i<8;i++) x[i]=threadIdx.x*8+i+s;
  for (int r=0;r<R;r++){
#pragma unroll
    for (int i=0;i<8;i++) x[i]=__builtin_amdgcn_alignbit(x[i], x[(i+1)&7], 9u + (uint32_t)i); }
  uint32_t a=0; for(int i=0;i<8;i++) a^=x[i];
  out[blockIdx.x*blockDim.x+threadIdx.x]=a;
}
// mixes: 8 chains of each of two instruction types per iteration (16 ops)
__global__ void k_mix_bitop3_fma32(float* out, float s) {
  uint32_t x[8]; float y[8];
  for (int i=0;i<8;i++){ x[i]=threadIdx.x*8+i+(uint32_t)s; y[i]=threadIdx.x*1e-3f+i+s; }
  for (int r=0;r<R;r++){
#pragma unroll
    for (int i=0;i<8;i++){ x[i]=__builtin_amdgcn_bitop3_b32(x[i], x[(i+1)&7], 7u+i, 0x96);
                           y[i]=__builtin_fmaf(y[i], 0.999f, 0.001f); } }
  float a=0; for(int i=0;i<8;i++) a+=y[i]+(float)(x[i]&1u);
  out[blockIdx.x*blockDim.x+threadIdx.x]=a;
}
__global__ void k_mix_bitop3_mad(uint32_t* out, uint32_t s) {
  uint32_t x[8]; uint64_t p[8];
  for (int i=0;i<8;i++){ x[i]=threadIdx.x*8+i+s; p[i]=threadIdx.x*8+i+s+((uint64_t)blockIdx.x<<32); }
  for (int r=0;r<R;r++){
#pragma unroll
    for (int i=0;i<8;i++){ x[i]=__builtin_amdgcn_bitop3_b32(x[i], x[(i+1)&7], 7u+i, 0x96);
                           p[i]=(uint64_t)(uint32_t)p[i]*0xD2511F53u + p[i]; } }
  uint32_t a=0; for(int i=0;i<8;i++) a^=x[i]^(uint32_t)p[i]^(uint32_t)(p[i]>>32);
  out[blockIdx.x*blockDim.x+threadIdx.x]=a;
}
__global__ void k_mix_bitop3_fma64(double* out, double s) {
  uint32_t x[8]; double y[8];
  for (int i=0;i<8;i++){ x[i]=threadIdx.x*8+i+(uint32_t)s; y[i]=threadIdx.x*1e-3+i+s; }
  for (int r=0;r<R;r++){
#pragma unroll
    for (int i=0;i<8;i++){ x[i]=__builtin_amdgcn_bitop3_b32(x[i], x[(i+1)&7], 7u+i, 0x96);
                           y[i]=fma(y[i], 0.999, 0.001); } }
  double a=0; for(int i=0;i<8;i++) a+=y[i]+(double)(x[i]&1u);
  out[blockIdx.x*blockDim.x+threadIdx.x]=a;
}
template <typename T, typename K>
void run(const char* name, K kern, int ops_per_iter, int instrs_per_op) {
  const int blocks=256*16, threads=256;
  T* out; hipMalloc(&out, sizeof(T)*blocks*threads);
  hipEvent_t a,b; hipEventCreate(&a); hipEventCreate(&b);
  hipLaunchKernelGGL(kern, dim3(blocks), dim3(threads), 0, 0, out, (T)1);
  hipDeviceSynchronize();
  hipEventRecord(a);
  for (int it=0; it<5; ++it) hipLaunchKernelGGL(kern, dim3(blocks), dim3(threads), 0, 0, out, (T)1);
  hipEventRecord(b); hipEventSynchronize(b);
  float ms; hipEventElapsedTime(&ms, a, b);
  double ops = 5.0*blocks*threads*(double)R*ops_per_iter;
  printf("%-18s %8.3f ms  %.3e ops/s  = %.3f lane-ops/clk/CU (256 CU, 2.4 GHz)\n", name, ms, ops/(ms*1e-3),
         ops/(ms*1e-3)/(256*2.4e9));
  hipFree(out);
}
int main(){
  hipDeviceProp_t p; hipGetDeviceProperties(&p, 0);
  printf("device %s CUs %d clock %d kHz\n", p.gcnArchName, p.multiProcessorCount, p.clockRate);
  run<uint32_t>("mad_u64", k_mad, 8, 1);
  run<uint32_t>("philox/8", k_philox, 1, 1);
  run<uint32_t>("bitop3", k_bitop3, 8, 1);
  run<float>("fma_f32", k_fma32, 8, 1);
  run<double>("fma_f64", k_fma64, 8, 1);
  run<float>("sin_f32", k_sin, 8, 1);
  run<float>("exp_f32", k_exp, 8, 1);
  run<double>("cvtadd64", k_add64, 8, 1);
  run<uint32_t>("alignbit", k_alignbit, 8, 1);
  run<float>("mix:bitop3+fma32", k_mix_bitop3_fma32, 16, 1);
  run<uint32_t>("mix:bitop3+mad64", k_mix_bitop3_mad, 16, 1);
  run<double>("mix:bitop3+fma64", k_mix_bitop3_fma64, 16, 1);
  return 0;
}
