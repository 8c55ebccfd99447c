/*
 * ooc_kernels.h -- kernel ids accepted by ooc_par_loop, with the argument list
 * each expects (DAT arguments first, in this order; then CONST, DEVSCALAR and
 * RED arguments).  "R", "W", "RW" give the access mode; stencils are the
 * caller's, but must cover what the kernel reads (listed here).
 *
 * Offsets are (dx, dy[, dz]).  "4n" = the four nodes of a cell
 * {(0,0),(1,0),(0,1),(1,1)}; "4c" = the four cells of a node
 * {(-1,-1),(0,-1),(-1,0),(0,0)}.
 */
#ifndef OOC_KERNELS_H
#define OOC_KERNELS_H

enum {
  /* ---- generic ---- */
  /* n pairs (W dst_k @0, R src_k @o_k), n CONST sign_k: dst_k = sign_k * src_k(p + o_k).
   * Used for reflective-wall strips and field copies.  1 <= n <= 6. */
  OOC_K_MIRROR = 1,
  /* W dst @0, CONST value: dst = value */
  OOC_K_FILL = 2,
  /* R a_1..a_m @0 (1 <= m <= 3), RED(SUM): red += prod_k a_k */
  OOC_K_SUM_PROD = 3,
  /* W out @0, R in @{o_1..o_n}, CONST c0, CONST c1: out = c0 * mean_k in(p+o_k) + c1 */
  OOC_K_AVG = 4,
  /* INC out @0, R in @0, CONST c: out += c * in */
  OOC_K_INC_ADD = 5,
  /* R a @0, RED(MIN), RED(MAX): min / max of a */
  OOC_K_MINMAX = 6,

  /* ---- 2D hydro proxy (x = axis 0, y = axis 1; tiled along y) ---- */
  /* R rho, R e, W p, W cs: p = (g-1) rho e; cs = sqrt(g p / rho) */
  OOC_K_H2D_EOS = 100,
  /* R rho, R e, W p */
  OOC_K_H2D_EOS_P = 101,
  /* R rho0, R cs, R u0 4n, R v0 4n, W q */
  OOC_K_H2D_VISC = 102,
  /* R rho0, R e0, R p, R q, R vol, R xarea {(0,0),(1,0)}, R yarea {(0,0),(0,1)},
   * R u0 4n, R v0 4n, W rho1, W e1; DEVSCALAR dt */
  OOC_K_H2D_PDV_PRED = 103,
  /* as PDV_PRED plus R u1 4n, R v1 4n after v0 */
  OOC_K_H2D_PDV_CORR = 104,
  /* R rho0 4c, R vol 4c, R p 4c, R q 4c, R xarea {(0,-1),(0,0)}, R yarea {(-1,0),(0,0)},
   * R u0, R v0, W u1, W v1; CONST nx, CONST ny; DEVSCALAR dt */
  OOC_K_H2D_ACCEL = 105,
  /* R xarea, R u0 {(0,0),(0,1)}, R u1 {(0,0),(0,1)}, W vfx; DEVSCALAR dt */
  OOC_K_H2D_FLUX_X = 106,
  /* R yarea, R v0 {(0,0),(1,0)}, R v1 {(0,0),(1,0)}, W vfy; DEVSCALAR dt */
  OOC_K_H2D_FLUX_Y = 107,
  /* R vol, R vfx {(0,0),(1,0)}, R vfy {(0,0),(0,1)}, W pre, W post */
  OOC_K_H2D_ADV_VOL_X = 108,
  /* R vol, R vfy {(0,0),(0,1)}, W pre, W post */
  OOC_K_H2D_ADV_VOL_Y = 109,
  /* R vf, R rho1 {-e,0}, R e1 {-e,0}, W mf, W ef  (e = unit vector of the sweep) */
  OOC_K_H2D_ADV_FLUX_X = 110,
  OOC_K_H2D_ADV_FLUX_Y = 111,
  /* RW rho1, RW e1, R pre, R post, R mf {0,+e}, R ef {0,+e} */
  OOC_K_H2D_ADV_CELL_X = 112,
  OOC_K_H2D_ADV_CELL_Y = 113,
  /* R mf (x: {(0,-1),(0,0),(1,-1),(1,0)}; y: {(-1,0),(0,0),(-1,1),(0,1)}), W nf */
  OOC_K_H2D_NFLUX_X = 114,
  OOC_K_H2D_NFLUX_Y = 115,
  /* R rho1 4c, R post 4c, R nf {-e,0}, W nmpost, W nmpre */
  OOC_K_H2D_NMASS_X = 116,
  OOC_K_H2D_NMASS_Y = 117,
  /* R nf, R vel {0,+e}, W mflux */
  OOC_K_H2D_MFLUX_X = 118,
  OOC_K_H2D_MFLUX_Y = 119,
  /* RW vel, R nmpre, R nmpost, R mflux {-e,0} */
  OOC_K_H2D_VEL_X = 120,
  OOC_K_H2D_VEL_Y = 121,
  /* R e0, R u0 4n, R v0 4n; CONST dx, CONST dy; RED(MIN) dt */
  OOC_K_H2D_DT = 122,
  /* Field summary (interior range): R vol, R rho0, R e0, R u0 4n, R v0 4n;
   * RED(SUM) x5: volume = sum vol, mass = sum m (m = rho0 vol), internal
   * energy = sum m e0, kinetic energy = sum m w / 2 (w = mean of u0^2 + v0^2
   * over the 4 nodes), pressure = sum p vol (p = (gamma - 1) rho0 e0) */
  OOC_K_H2D_SUMMARY = 123,

  /* ---- 3D Navier-Stokes proxy (tiled along z).  q = conserved (rho, rho u,
   * rho v, rho w, rho E); prims = (rho, u, v, w, p); grads = du/dx, du/dy,
   * du/dz, dv/dx, ..., dw/dz, dT/dx, dT/dy, dT/dz.  "S" = the 12-point star
   * {(+-1,0,0),(+-2,0,0),(0,+-1,0),(0,+-2,0),(0,0,+-1),(0,0,+-2)}. ---- */
  /* R prims x5, W q x5 */
  OOC_K_NS_INIT = 200,
  /* R q x5, W prims x5 */
  OOC_K_NS_PRIMS = 201,
  /* R rho S, R u S, R v S, R w S, R p S, W grads x12; CONST 1/(12h), CONST gamma M^2 */
  OOC_K_NS_GRADS = 202,
  /* R prims x5 S, R grads x12 S, RW q x5, W dq x5 (first stage) or RW dq x5;
   * CONST 1/(12h), mu, kappa, dt, A_s, B_s: dq = A_s dq + dt R(q); q += B_s dq */
  OOC_K_NS_RHS_FIRST = 203,
  OOC_K_NS_RHS = 204,
  /* The same residual + update with the gradients evaluated from the
   * primitives inside the kernel (no stored gradient fields):
   * R prims x5 G, RW q x5, W dq x5 (first stage) or RW dq x5;
   * CONST 1/(12h), mu, kappa, dt, A_s, B_s, gamma M^2.  "G" = the 73 points
   * {a e_A + b e_B : a, b in {0, +-1, +-2}; axes A, B} (fluxes at the points of
   * the 5-point stencils, each from the 5-point stencils of the primitives). */
  OOC_K_NS_RHS_FUSED_FIRST = 205,
  OOC_K_NS_RHS_FUSED = 206,
  /* The same with the primitives evaluated from the conserved variables
   * inside the kernel too (no primitives loop, no primitive fields), reading
   * one copy of the conserved variables and writing the other:
   * R q x5 G, W q' x5, W dq x5 (first stage) or RW dq x5; the same CONSTs:
   * dq = A_s dq + dt R(q); q' = q + B_s dq. */
  OOC_K_NS_RHS_FUSEDQ_FIRST = 207,
  OOC_K_NS_RHS_FUSEDQ = 208,

  /* ---- 3D hydro proxy (tiled along z).  "8n" = the 8 nodes of a cell
   * {0,1}^3; "8c" = the 8 cells of a node {-1,0}^3; "F4x" = the 4 nodes of a
   * cell's x-face {(e,0,0),(e,1,0),(e,0,1),(e,1,1)} (likewise y, z); e_D = the
   * unit vector of sweep D.  EOS / EOS_P of the 2D proxy are point-wise and
   * serve in 3D unchanged. ---- */
  /* R rho0, R cs, R u0 8n, R v0 8n, R w0 8n, W q */
  OOC_K_H3D_VISC = 300,
  /* R rho0, R e0, R p, R q, R vol, R xarea {0,+x}, R yarea {0,+y}, R zarea {0,+z},
   * R u0 8n, R v0 8n, R w0 8n, W rho1, W e1; DEVSCALAR dt */
  OOC_K_H3D_PDV_PRED = 301,
  /* as PDV_PRED plus R u1 8n, R v1 8n, R w1 8n after w0 */
  OOC_K_H3D_PDV_CORR = 302,
  /* R rho0 8c, R vol 8c, R p 8c, R q 8c, R xarea {(0,b,c)}, R yarea {(a,0,c)},
   * R zarea {(a,b,0)} (a, b, c in {-1,0}), R u0, R v0, R w0, W u1, W v1, W w1;
   * CONST nx, ny, nz; DEVSCALAR dt */
  OOC_K_H3D_ACCEL = 303,
  /* R area, R vel0 F4, R vel1 F4, W vf; DEVSCALAR dt (vel = u for x, v for y, w for z) */
  OOC_K_H3D_FLUX_X = 304,
  OOC_K_H3D_FLUX_Y = 305,
  OOC_K_H3D_FLUX_Z = 306,
  /* X: R vol, R vfx {0,+x}, R vfy {0,+y}, R vfz {0,+z}, W pre, W post
   * Y: R vol, R vfy, R vfz, W pre, W post;  Z: R vol, R vfz, W pre, W post */
  OOC_K_H3D_ADV_VOL_X = 307,
  OOC_K_H3D_ADV_VOL_Y = 308,
  OOC_K_H3D_ADV_VOL_Z = 309,
  /* R vf, R rho1 {-e_D,0}, R e1 {-e_D,0}, W mf, W ef */
  OOC_K_H3D_ADV_FLUX_X = 310,
  OOC_K_H3D_ADV_FLUX_Y = 311,
  OOC_K_H3D_ADV_FLUX_Z = 312,
  /* RW rho1, RW e1, R pre, R post, R mf {0,+e_D}, R ef {0,+e_D} */
  OOC_K_H3D_ADV_CELL_X = 313,
  OOC_K_H3D_ADV_CELL_Y = 314,
  OOC_K_H3D_ADV_CELL_Z = 315,
  /* R mf {e e_D - b e_B - c e_C : e, b, c in {0,1}} (B, C the other two axes), W nf */
  OOC_K_H3D_NFLUX_X = 316,
  OOC_K_H3D_NFLUX_Y = 317,
  OOC_K_H3D_NFLUX_Z = 318,
  /* R rho1 8c, R post 8c, R nf {-e_D,0}, W nmpost, W nmpre */
  OOC_K_H3D_NMASS_X = 319,
  OOC_K_H3D_NMASS_Y = 320,
  OOC_K_H3D_NMASS_Z = 321,
  /* R nf, R vel {0,+e_D}, W mflux */
  OOC_K_H3D_MFLUX_X = 322,
  OOC_K_H3D_MFLUX_Y = 323,
  OOC_K_H3D_MFLUX_Z = 324,
  /* RW vel, R nmpre, R nmpost, R mflux {-e_D,0} */
  OOC_K_H3D_VEL_X = 325,
  OOC_K_H3D_VEL_Y = 326,
  OOC_K_H3D_VEL_Z = 327,
  /* R e0, R u0 8n, R v0 8n, R w0 8n; CONST dx, dy, dz; RED(MIN) dt */
  OOC_K_H3D_DT = 328,

  OOC_K_MAX_ID = 512
};

#endif /* OOC_KERNELS_H */
