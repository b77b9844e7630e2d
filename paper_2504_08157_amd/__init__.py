"""MI355X (gfx950) hot path of an element-based Galerkin nonhydrostatic
model: hand-written HIP kernels behind the C ABI of include/nhsem.h.

  csrc/nh_kernels.hip  fused RHS + DSS + SSP-RK stage kernel (FP64 and
                       FP32-mixed), batched form, DSS/scatter/mass/diagnostics
  csrc/nh_hevi.hip     vertical operator L_v and the column GMRES solvers
  csrc/nh_mlp.hip      column MLP: features, FP16-MFMA GEMMs, fused inference
  csrc/nh_hyper.hip    tensor hyper-diffusion (directional weak Laplacian)
  csrc/nh_imex3d.hip   3D linear operator and the global GMRES of 3D-IMEX
  csrc/nh_ri.hip       RI-velocity diagnostic
  csrc/nhsem.cpp       host layer: contexts, workspaces, steppers, C ABI
  nhsem.py             ctypes binding (argument marshalling only)
  build.py             in-tree build of libnhsem.so with hipcc
  workloads.py         synthetic workload definitions shared with the tests
  learned_guess.py     training and evaluation of the column-MLP guess
"""
