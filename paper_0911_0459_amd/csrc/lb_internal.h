// Internal types shared by the host runtime and the HIP kernels of lbcap.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lbcap.h"

namespace lbk {

// Records the message returned by lb_last_error and returns s.
lb_status set_error(lb_status s, const char* msg);

constexpr int TILE_W = 64;  // tile width along x = one wavefront

// Per-capillary descriptor, resident in device memory.  Offsets are in floats
// from the base of each arena (the two arenas have identical layout).
//
// Stored per capillary and arena, each plane ny x pitch floats:
//   planes 0..8   s_i = f_i - r_i, the shifted post-collision populations
//                 (moment storage, binary: planes 0..6 hold the seven numbers
//                 that fix them instead, see lb_wmom.h)
//   plane  9      phi (binary only): the order parameter, in 32-bit fixed point
//                 (29 fraction bits) in the plane's bits
// A step reads arena `cur ^ par` and writes the other one.  After step t the
// read-from arena of the next step holds f*(t) and phi(t+1), and the other
// arena's plane 9 still holds phi(t).
struct CapDev {
    int nx, ny, pitch;       // lattice size; row pitch in floats (multiple of 64)
    int x_in, x_end;         // tube columns [x_in, x_end)
    int y0, y1;              // tube fluid rows [y0, y1)
    int active;              // 0: retired, not advanced
    int par;                 // this capillary reads arena cur ^ par
    int mstore;              // 1: moment storage (planes 0..6 hold the post-collision state), else 9 populations
    long long off_f;         // offset of plane 0
    long long off_phi;       // offset of the phi plane (binary)
    long long plane;         // floats per plane = ny * pitch
    float kappa, a, b, T;    // vdW constants
    float A, B, Gamma;       // binary constants
    float nu_l, nu_g;        // viscosities
    float omega_l;           // 2/(6 nu_l + 1)
    float G;                 // wall gradient (normal into fluid)
    float Fx;                // body force
    float lam_on;            // 1: vdW Galilean lambda active
    float q_mid;             // interface level
    // Reference rest state subtracted from the stored f populations:
    // s_i = f_i - r_i with r the equilibrium at density rho_ref, u = 0, no
    // gradients (r_0 = rho_ref - 5/3 X_ref, axis X_ref/3, diagonal X_ref/12).
    float rho_ref;           // vdW: mid density; binary: 1
    float X_ref;             // bulk pressure of the reference state
    float ibr;               // vdW: 1/(1 - b rho_ref)
    float phib2;             // binary: bulk phi^2 = A/B
    int hist_off;            // offset of this capillary's history in the history arrays
    float phib;              // binary: bulk phi = sqrt(A/B)
};

// One tile: capillary index, tile origin, number of rows inside the lattice.
struct TileDev {
    int cap, x0, y0, rows;
};

struct StepArgs {
    const CapDev* caps;
    const TileDev* tiles;
    int ntiles;
    int schedule;            // 0 linear, 1 XCD-grouped, 2 persistent stride
    float* arena0;
    float* arena1;
    int cur;                 // capillary k reads arena (cur ^ par_k), writes the other
    int init;                // 1: initialisation from the field in the read arena
};

}  // namespace lbk
