"""MI355X-native (gfx950) HLBM mean-flow adjoint: primal HLBM sweep, FP64
window averaging, adjoint LBM sweep and porosity gradient, behind the C ABI
of libhlbm.so (include/hlbm.h).  The Python modules only marshal arguments."""
