"""MI355X (gfx950) hot path of the finite-difference micromagnetic method of
MicroMagnetic.jl (arXiv 2406.16064): effective field (Newell-tensor FFT demag,
exchange, interfacial DMI, uniaxial anisotropy, Zeeman), Landau-Lifshitz
right-hand side and adaptive Dormand-Prince integration, behind the C interface
include/mm.h.  `paper_2406_16064_amd.mm` is the ctypes binding (it raises on
import when libmmx.so is missing); `paper_2406_16064_amd.inputs` holds the
seeded synthetic inputs.
"""
