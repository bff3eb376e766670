// Two time steps per launch (temporal blocking) for the FP32 step on
// periodic grids: k_step2 takes the state at step n from HBM and writes the
// state at step n + 2, keeping the intermediate state n + 1 on chip.  Each
// step is the same arithmetic as k_step_fused (phi of Sec. 2.3.1, eq.
// order-parameter; mu of Sec. 2.1, eq. chemical_potencial; the collisions of
// Secs. 2.3.1-2.3.2 through cell_f32), so the result is bit-identical to two
// single steps; only the population planes of every second step travel
// through HBM.
//
// A workgroup owns a strip of W output columns (W + 10 <= 256, a kernel
// argument) and H output rows and marches up it.  Lane l stands for column x0 - 5 + l (periodic wrap) in
// every role:
//   step A (n -> n + 1): phi on lanes [0, W + 10), mu on [1, W + 9), the
//     collision on [2, W + 8), i.e. on the strip plus three columns each side;
//   step B (n + 1 -> n + 2): phi on [3, W + 7), mu on [4, W + 6), the
//     collision on [5, W + 5), the strip itself.
// Step A runs four rows ahead of step B (B's collision at row y needs A's
// output on rows y - 3 .. y + 3).  A's output rows stay in the registers of
// the lane that computed them; each row, every lane stages the few values
// the pull gathers of step B read from its neighbours into LDS (f for B's phi
// of one row, g for B's collision of another), so no full intermediate row
// of 19 planes is held anywhere.  Step A's own gathered f waits in an LDS
// ring of three rows between its phi and its collision.  S (u . grad phi) of step n + 2 goes to a
// second S plane: step A needs S_prev of step n on the halo cells, which the
// strips beside it would otherwise overwrite.
#pragma once
#include "forward.h"

namespace lbm {

constexpr int S2_L = 256;  // lanes per workgroup
constexpr int S2_WMAX = S2_L - 10;  // widest strip: step A's phi takes W + 10 lanes
constexpr int S2_H = 128;  // tallest strip; the host may lower it

__device__ __forceinline__ int wrap_row(int v, int n) { return stencil_idx(v, n, 0); }

// Directions by the row they are pulled from: cy = -1 (4 S, 7 SW, 8 SE) from
// the row above, cy = 0 (0, 1 E, 3 W) from the same row, cy = +1 (2 N, 5 NE,
// 6 NW) from the row below.
template <typename F>
__device__ __forceinline__ void for_dirs_cy(int cy, F&& f) {
  if (cy == -1) { f(4); f(7); f(8); }
  if (cy == 0) { f(0); f(1); f(3); }
  if (cy == 1) { f(2); f(5); f(6); }
}

template <bool MRT, bool NT, bool LO16>
__global__ __launch_bounds__(S2_L, 2) void k_step2(const KP p, const float* Bin, float* Bout,
                                                   const float* Sin, float* Sout, int W, int ntx,
                                                   int H, int xcd_order) {
  __shared__ float phA[5][S2_L];   // phi - phi_ref of step A, by lane
  __shared__ float muA[3][S2_L];
  __shared__ float phB[5][S2_L];   // of step B
  __shared__ float muB[3][S2_L];
  __shared__ float SF[10][S2_L];   // A's f_0..f_8 and low word, for B's phi gather
  __shared__ float SG[2][9][S2_L]; // A's g, for B's collision gather (two rows in turn)
  __shared__ float FA[3][10][S2_L]; // step A's gathered f of rows k, k+1, k+2 (by row mod 3)

  const int blk = xcd_order ? xcd_tile(blockIdx.x, gridDim.x) : (int)blockIdx.x;
  const int x0 = (blk % ntx) * W, y0 = (blk / ntx) * H;
  const int y1 = y0 + H < p.ny ? y0 + H : p.ny;
  const int l = threadIdx.x;
  const int cu = x0 - 5 + l;  // unwrapped column of this lane
  const int xc = stencil_idx(cu, p.nx, 0);
  const int xm = stencil_idx(cu - 1, p.nx, 0), xp = stencil_idx(cu + 1, p.nx, 0);
  unsigned bxc = 4u * (unsigned)xc, bxm = 4u * (unsigned)xm, bxp = 4u * (unsigned)xp;
  const bool rPhiA = l < W + 10, rMuA = l >= 1 && l < W + 9, rColA = l >= 2 && l < W + 8;
  const bool rPhiB = l >= 3 && l < W + 7, rMuB = l >= 4 && l < W + 6;
  const bool rColB = l >= 5 && l < W + 5 && cu < p.nx;
  const long long ps = p.ps;
  const int pitch = p.pitch;
  // the buffers, made opaque once per row below: the compiler then forms
  // each plane's base next to its access (scalar arithmetic) instead of
  // keeping some forty 64-bit plane bases live across the loop, which it
  // cannot hold in scalar registers without spilling them
  const float* Bi = Bin;
  float* Bo = Bout;
  const float* Si = Sin;
  float* So = Sout;

  // byte offset of the pull source column of direction i
  auto colb = [&](int i) { return cx_of(i) == 1 ? bxm : (cx_of(i) == -1 ? bxp : bxc); };
  // f_0..f_8 and the low word of f_0 pulled to (this lane's column, row r)
  auto gather_f = [&](int r, float (&f)[10]) {
    const int ym = wrap_row(r - 1, p.ny), yc = wrap_row(r, p.ny), yp = wrap_row(r + 1, p.ny);
#pragma unroll
    for (int i = 0; i < 9; ++i) {
      const int sy = cy_of(i) == 1 ? ym : (cy_of(i) == -1 ? yp : yc);
      f[i] = ld_at(Bi + i * ps + (long long)sy * pitch, colb(i));
    }
    if constexpr (LO16)
      f[9] = lo_decode(f[0], ld_at(lo_plane(Bi, p) + (long long)yc * pitch, bxc >> 1));
    else
      f[9] = ld_at(Bi + LO_PLANE * ps + (long long)yc * pitch, bxc);
  };
  auto gather_g = [&](int r, float (&g)[9], float& Sp) {
    const int ym = wrap_row(r - 1, p.ny), yc = wrap_row(r, p.ny), yp = wrap_row(r + 1, p.ny);
#pragma unroll
    for (int i = 0; i < 9; ++i) {
      const int sy = cy_of(i) == 1 ? ym : (cy_of(i) == -1 ? yp : yc);
      g[i] = ld_at(Bi + (9 + i) * ps + (long long)sy * pitch, colb(i));
    }
    Sp = ld_at(Si + (long long)yc * pitch, bxc);
  };
  auto phi_of = [&](const float (&f)[10]) {
    Pops<float> q;
#pragma unroll
    for (int i = 0; i < 9; ++i) q.f[i] = f[i];
    q.lo = f[9];
    return phi_sum<float>(q);
  };
  auto mu_at = [&](float (*ph)[S2_L], int r) {
    const float* r0 = ph[mod_pos(r - 1, 5)];
    const float* r1 = ph[mod_pos(r, 5)];
    const float* r2 = ph[mod_pos(r + 1, 5)];
    const float v[3][3] = {{r0[l - 1], r0[l], r0[l + 1]}, {r1[l - 1], r1[l], r1[l + 1]},
                           {r2[l - 1], r2[l], r2[l + 1]}};
    return mu_cell<float>(p, v);
  };
  auto nbhd_at = [&](float (*ph)[S2_L], float (*mu)[S2_L], int r, Nbhd<float>& nb) {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const float* pr = ph[mod_pos(r - 1 + a, 5)];
      const float* mr = mu[mod_pos(r - 1 + a, 3)];
#pragma unroll
      for (int b = 0; b < 3; ++b) {
        nb.ph[a][b] = pr[l - 1 + b];
        nb.mu[a][b] = mr[l - 1 + b];
      }
    }
  };

  // step B's gathered f of rows k-4, k-3 (k-2 arrives in the iteration)
  float fb0[10], fb1[10];
  // Step A's output by age (rows k-1, k-2, ... at the top of iteration k):
  // f at ages 1-3, g at ages 1-5, S at ages 1-4.  Ages past a value's last
  // use are not kept (f: age 2 keeps cy >= 0, age 3 cy = +1; g: age 4 keeps
  // cy >= 0, age 5 cy = +1); indices stay those of the directions.
  float af1[10], af2[10], af3[10];
  float ag1[9], ag2[9], ag3[9], ag4[9], ag5[9];
  float aS1 = 0.f, aS2 = 0.f, aS3 = 0.f, aS4 = 0.f;
#pragma unroll
  for (int i = 0; i < 10; ++i) af1[i] = af2[i] = af3[i] = 0.f;
#pragma unroll
  for (int i = 0; i < 9; ++i) ag1[i] = ag2[i] = ag3[i] = ag4[i] = ag5[i] = 0.f;
  // loads in flight: f of step A's next phi row, g and S_prev of its next
  // collision row
  float fN[10], gN[9], SN;

  // prologue: phi_A of rows y0-5 .. y0-2, mu_A of rows y0-4, y0-3
  for (int r = y0 - 5; r <= y0 - 2; ++r) {
    float f[10];
    if (rPhiA) {
      gather_f(r, f);
      phA[mod_pos(r, 5)][l] = phi_of(f);
    }
    if (r >= y0 - 3 && rColA) {
#pragma unroll
      for (int i = 0; i < 10; ++i) FA[mod_pos(r, 3)][i][l] = f[i];
    }
  }
  __syncthreads();
  if (rMuA) {
    muA[mod_pos(y0 - 4, 3)][l] = mu_at(phA, y0 - 4);
    muA[mod_pos(y0 - 3, 3)][l] = mu_at(phA, y0 - 3);
  }
  if (rPhiA) gather_f(y0 - 1, fN);
  if (rColA) gather_g(y0 - 3, gN, SN);

  for (int kk = y0 - 3; kk <= y1 + 3; ++kk) {
    // the row counter is uniform; saying so keeps the row arithmetic and the
    // row addresses in scalar registers
    const int k = __builtin_amdgcn_readfirstlane(kk);
    // The column offsets, opaque once per row: the compiler then forms each
    // address as a scalar base plus a zero-extended 32-bit offset next to
    // its access (the scalar-base form of the global access) instead of
    // adding 64-bit vector sums hoisted out of the loop.
    asm volatile("" : "+v"(bxc), "+v"(bxm), "+v"(bxp));
    asm volatile("" : "+s"(Bi), "+s"(Bo), "+s"(Si), "+s"(So));
    const bool doA = k <= y1 + 2;
    // ---- P1: phi_A(k+2); stage A's output for B
    if (doA && rPhiA) {
      phA[mod_pos(k + 2, 5)][l] = phi_of(fN);
      if (rColA) {
#pragma unroll
        for (int i = 0; i < 10; ++i) FA[mod_pos(k + 2, 3)][i][l] = fN[i];
      }
      // the next row's f goes out at once: a whole iteration hides it
      if (k + 1 <= y1 + 2) gather_f(k + 3, fN);
    }
    if (rColA) {
      // B's phi of row k-2 pulls from A rows k-1 (cy = -1), k-2 (cy = 0), k-3 (cy = +1)
      for_dirs_cy(-1, [&](int i) { SF[i][l] = af1[i]; });
      for_dirs_cy(0, [&](int i) { SF[i][l] = af2[i]; });
      SF[9][l] = af2[9];
      for_dirs_cy(1, [&](int i) { SF[i][l] = af3[i]; });
      // B's collision at row k-4 pulls g from A rows k-3, k-4, k-5
      float(*sg)[S2_L] = SG[k & 1];
      for_dirs_cy(-1, [&](int i) { sg[i][l] = ag3[i]; });
      for_dirs_cy(0, [&](int i) { sg[i][l] = ag4[i]; });
      for_dirs_cy(1, [&](int i) { sg[i][l] = ag5[i]; });
    }
    __syncthreads();
    // ---- P2: mu_A(k+1); phi_B(k-2)
    if (doA && rMuA) muA[mod_pos(k + 1, 3)][l] = mu_at(phA, k + 1);
    float fb2[10];
    if (k >= y0 && rPhiB) {
#pragma unroll
      for (int i = 0; i < 9; ++i) fb2[i] = SF[i][l - cx_of(i)];
      fb2[9] = SF[9][l];
      phB[mod_pos(k - 2, 5)][l] = phi_of(fb2);
    }
    __syncthreads();
    // ---- P3: collision A at row k (then the next row's loads); mu_B(k-3)
    // A's output ages by one row; the new row becomes age 1
    for_dirs_cy(1, [&](int i) { af3[i] = af2[i]; });
    for_dirs_cy(0, [&](int i) { af2[i] = af1[i]; });
    for_dirs_cy(1, [&](int i) { af2[i] = af1[i]; });
    af2[9] = af1[9];
    for_dirs_cy(1, [&](int i) { ag5[i] = ag4[i]; });
    for_dirs_cy(0, [&](int i) { ag4[i] = ag3[i]; });
    for_dirs_cy(1, [&](int i) { ag4[i] = ag3[i]; });
#pragma unroll
    for (int i = 0; i < 9; ++i) {
      ag3[i] = ag2[i];
      ag2[i] = ag1[i];
    }
    float nS = 0.f;
    if (doA && rColA) {
      Pops<float> q;
      const float(*fk)[S2_L] = FA[mod_pos(k, 3)];
#pragma unroll
      for (int i = 0; i < 9; ++i) {
        q.f[i] = fk[i][l];
        q.g[i] = gN[i];
      }
      q.lo = fk[9][l];
      Nbhd<float> nb;
      nbhd_at(phA, muA, k, nb);
      CellOut c;
      float fo[9], lo = 0.f;
      cell_f32<true, MRT>(p, q, nb, SN, fo, lo, ag1, c);
#pragma unroll
      for (int i = 0; i < 9; ++i) af1[i] = fo[i];
      // the low word as a store and a reload would leave it
      af1[9] = LO16 ? lo_decode(fo[0], lo_encode(fo[0], lo)) : lo;
      nS = (float)c.S;
    }
    if (k + 1 <= y1 + 2 && rColA) gather_g(k + 1, gN, SN);
    if (k >= y0 + 2 && rMuB) muB[mod_pos(k - 3, 3)][l] = mu_at(phB, k - 3);
    __syncthreads();
    // ---- P4: collision B at row k-4, stored
    if (k >= y0 + 4 && rColB) {
      const int y = k - 4;
      const float(*sg)[S2_L] = SG[k & 1];
      Pops<float> q;
#pragma unroll
      for (int i = 0; i < 9; ++i) {
        q.f[i] = fb0[i];
        q.g[i] = sg[i][l - cx_of(i)];
      }
      q.lo = fb0[9];
      Nbhd<float> nb;
      nbhd_at(phB, muB, y, nb);
      CellOut c;
      float fo[9], go[9], lo = 0.f;
      cell_f32<true, MRT>(p, q, nb, aS4, fo, lo, go, c);
      const long long row = (long long)y * pitch;
#pragma unroll
      for (int i = 0; i < 9; ++i) {
        st_at<NT>(Bo + i * ps + row, bxc, fo[i]);
        st_at<NT>(Bo + (9 + i) * ps + row, bxc, go[i]);
      }
      if constexpr (LO16)
        st_at<NT>(lo_plane(Bo, p) + row, bxc >> 1, lo_encode(fo[0], lo));
      else
        st_at<NT>(Bo + LO_PLANE * ps + row, bxc, lo);
      st_at<NT>(So + row, bxc, (float)c.S);
    }
    // ---- the rings and S age by one row
#pragma unroll
    for (int i = 0; i < 10; ++i) {
      fb0[i] = fb1[i];
      fb1[i] = fb2[i];
    }
    aS4 = aS3;
    aS3 = aS2;
    aS2 = aS1;
    aS1 = nS;
  }
}

}  // namespace lbm
