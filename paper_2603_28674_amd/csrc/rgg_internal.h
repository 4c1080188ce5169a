// Internal declarations shared by librgg's own translation units (host build
// stage, kernels, C ABI).  Not installed; the public interface is rgg.h.
#pragma once

#include <stdint.h>

#include <string>
#include <vector>

#include "rgg.h"

namespace rgg {

constexpr int kMaxSpheres = 64;     // one wavefront covers every sphere of an edge
constexpr int kMaxLinks = 32;
constexpr int kAabbStride = 8;      // floats per edge box: lo[3], s, hi[3], pad
// configurations per edge: at least 2 (both ends, a node (v, v) included), at
// most 2^24 (the kernels index an edge's copies with 32-bit integers)
constexpr int64_t kMinEdgeConfigs = 2;
constexpr int64_t kMaxEdgeConfigs = (int64_t)1 << 24;

// Approximations of a range of edges, built on the host in binary64.
//
// Sphere samples of edge e occupy [soff[e], soff[e+1]) in "sphere-sample"
// units, P_e = soff[e+1] - soff[e] = B * J_e for J_e configurations.  The
// coordinates are stored per edge as a [B][J_e][S] block starting at index
// S*soff[e], S = copy_stride(D) (xyz and one pad value in 3-D, xy in 2-D):
// one copy is one aligned 16- or 8-byte load, the copies of one sphere along
// the edge are contiguous, and the spheres whose capsule missed are never
// read.
inline int copy_stride(int D) { return D == 3 ? 4 : 2; }

struct HostGeometry {
    int kind = 0, D = 0, B = 0;
    int64_t E = 0;
    std::vector<int64_t> soff;     // [E+1]
    std::vector<double> samp;      // [sum_e S*P_e], S = copy_stride(D)
    std::vector<double> cap;       // [E][2D+1][B]: A_0..A_{D-1}, B_0..B_{D-1}, R
    std::vector<float> aabb;       // [E][8]: padded FP32 box lo[3], s, hi[3], 0
    std::vector<double> radius;    // [B]
    // full validation: the robot and each edge's motion
    int dof = 0, L = 0;
    std::vector<double> rob_pos;   // SE2 [B][2], SE3 [B][3], arm [B]
    std::vector<int32_t> rob_link; // arm [B]
    std::vector<double> rob_len;   // arm [L]
    double rob_base[2] = {0.0, 0.0};
    std::vector<double> motion;    // [E][2 dof + 3]: a, b (SE3: short-arc sign), turn, half, sin_half
    std::vector<double> delta;     // [E][B] chord-deviation bounds delta_i
    // the second forms of Sec. 4.2, when asked for
    int n_bodies = 1;              // robot bodies: 1 (rigid kinds) or L (arm links)
    std::vector<int32_t> body;     // [B] body of each sphere
    std::vector<uint8_t> body_has; // [n_bodies] the body carries a sphere
    std::vector<double> obb;       // [E][n_bodies][2D + D*D] oriented boxes: centre, axes
                                   // (row k = axis k), half-extents; empty without them
    std::vector<int64_t> sseg;     // [E*B + 1] first spline segment of (edge, sphere); empty
                                   // without splines
    std::vector<double> seg;       // [segments][2D + 1] spline segments: A, B, rho
};
inline int obb_stride(int D) { return 2 * D + D * D; }
constexpr double kDefaultSplineTol = 0.05;

// Validates the inputs of rgg_build.  Returns RGG_OK or RGG_E_INVALID_ARG
// with *err describing the problem.
rgg_status validate_build_inputs(const rgg_roadmap_desc *rd, const rgg_robot *rob,
                                 const rgg_build_opts *opts, std::string *err);

// Builds the approximations of edges [e0, e1).  Inputs must be validated.
rgg_status build_geometry(const rgg_roadmap_desc *rd, const rgg_robot *rob,
                          const rgg_build_opts *opts, int64_t e0, int64_t e1, int threads,
                          HostGeometry *out, std::string *err);

// Uniform grid over the edge boxes (Sec. 4.3 spatially filtered checking).
struct HostGrid {
    int32_t dim[3] = {1, 1, 1};
    double org[3] = {0, 0, 0};
    double inv = 0.0;              // 1 / cell size; 0 = a single cell
    double cell = 0.0;
    std::vector<int32_t> start;    // [ncells+1]
    std::vector<int32_t> edges;    // edge ids per cell, ascending
    int64_t items_cap = 0;         // sum over cells of max(1, ceil(n/chunk))
    // Block-local slab masks of the item kernel: local_slabs(D) slabs per
    // axis over the same bounds, in binary32.
    float sl_org[3] = {0, 0, 0};
    float sl_inv[3] = {0, 0, 0};   // slabs per unit length; 0: one slab
};

// Slabs per axis of the slab masks (slabs_of of the device header).
constexpr int local_slabs(int D) { return D == 3 ? 80 : 128; }

// Cell of coordinate x: floor((x - org) * inv), as an integer in [-1, n]
// (-1 below the grid, n above it).  The device evaluates the same binary64
// expression, so registration and lookup agree and are monotone in x.
int32_t cell_coord(double x, double org, double inv, int32_t n);

rgg_status build_grid(const HostGeometry &g, double cell_size, int32_t chunk, HostGrid *out,
                      std::string *err);

// Rounds a binary64 value to binary32 toward -inf / +inf.
float f32_down(double x);
float f32_up(double x);

}  // namespace rgg
