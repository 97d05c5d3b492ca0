// Internal interface between the host API and the kernel launchers.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lbm_common.hpp"

namespace tplbm {

// Everything one lattice launch needs.
struct LatticeLaunch {
    const void *fin;
    void *fout;
    const double *Tin;
    double *Tout;
    Phys phys;
    int nx, ny, nz;
    bool fp32, tau1, walls;
    bool moments;         // the state is moments (D2Q9: rho, j_x, j_y; D3Q19: rho, j and the readout's psi plane), not populations
    int resident;         // blocks of the persistent grid (two per compute unit)
    double *partials;     // 5 doubles per block
    StepState *st;
    int64_t step;         // level the launch starts from
    hipStream_t stream;
    const double *rref;   // FP32 deviations: reference density per wall-normal layer
};

// Velocity set of a lattice for the per-layer reference kernels: weights and
// the wall-normal velocity component of each population.
struct LayerSet {
    int Q;
    double w[19];
    int cn[19];
};

// Re-centre the FP32 deviations of every wall-normal layer (lnodes nodes
// each, nlayers of them) on the layer's current mean density, then write the
// level's <rho> and mass into st (parity slot `slot`).  lmass: nlayers doubles.
hipError_t recentre_layers_launch(float *f, double *rref, double *lmass, size_t N, int lnodes, int nlayers,
                                  const LayerSet &q, bool walls, StepState *st, int slot, hipStream_t s);

// D3Q19 velocity set of this library: rest, +x -x +y -y +z -z, 12 edges
constexpr int kD3Q19x[19] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
constexpr int kD3Q19y[19] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1};
constexpr int kD3Q19z[19] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1};

int d2q9_num_blocks(int nx, int ny, int resident, bool moments = false);
int d3q19_num_blocks(int nx, int ny, int nz, int cus);
hipError_t d3q19_launch_step(const LatticeLaunch &L, double *U);
hipError_t d3q19_launch_readout(const LatticeLaunch &L, int field, double *M, double *U, double *out);
// psi plane of a level-0 moment state M (rho and j set) from rho and L.Tin
hipError_t d3q19_launch_psi_init(const LatticeLaunch &L, double *M);
// D3Q19 update by z marching (d3q19_march.hip), population or moment state;
// U holds at least 4 planes of N doubles (u and rho of the level, handed
// from the LBM kernel to the energy kernel)
int d3q19_march_blocks(int nx, int ny, int nz, int cus);
hipError_t d3q19_march_step(const LatticeLaunch &L, double *U);
hipError_t d2q9_launch_step(const LatticeLaunch &L);
// moment-state D2Q9 update by row marching (d2q9_march.hip)
int d2q9_march_blocks(int nx, int ny, int cus);
hipError_t d2q9_march_launch(const LatticeLaunch &L);
hipError_t d2q9_launch_readout(const LatticeLaunch &L, int field, double *scratch, double *out);

}  // namespace tplbm
