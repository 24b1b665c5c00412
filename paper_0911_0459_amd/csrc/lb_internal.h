// Internal types shared by the host runtime and the HIP kernels of lbcap.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lbk {

constexpr int TILE_W = 64;  // tile width along x = one wavefront

// Per-capillary descriptor, resident in device memory.  Offsets are in floats
// from the base of each population arena (the two arenas have identical layout).
struct CapDev {
    int nx, ny, pitch;       // lattice size; row pitch in floats (multiple of 64)
    int x_in, x_end;         // tube columns [x_in, x_end)
    int y0, y1;              // tube fluid rows [y0, y1)
    int active;              // 0: retired, not advanced
    long long off_f;         // offset of f plane 0
    long long off_g;         // offset of g plane 0 (binary)
    long long plane;         // floats per plane = ny * pitch
    float kappa, a, b, T;    // vdW constants
    float A, B, Gamma;       // binary constants
    float nu_l, nu_g;        // viscosities
    float omega_l;           // 2/(6 nu_l + 1)
    float G;                 // wall gradient (normal into fluid)
    float Fx;                // body force
    float lam_on;            // 1: vdW Galilean lambda active
    float q_mid;             // interface level
    int hist_off;            // offset of this capillary's history in the history arrays
    int pad0;
};

// One tile: capillary index and tile origin.
struct TileDev {
    int cap, x0, y0, rows;
};

struct StepArgs {
    const CapDev* caps;
    const TileDev* tiles;
    int ntiles;
    int schedule;            // 0 linear, 1 XCD-grouped, 2 persistent stride
    const float* src;        // populations f*(t-1) (and g*)
    float* dst;              // populations f*(t)
    const float* init_q;     // INIT only: initial field of capillary k as ny*nx floats at caps[k].off_f
};

}  // namespace lbk
