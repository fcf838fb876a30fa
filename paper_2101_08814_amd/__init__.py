"""MI355X (gfx950) implementation of the SOAP hot path of Musil et al.,
"Efficient implementation of atom-density representations" (arXiv 2101.08814):
neighbour list, spherical expansion with splined GTO radial integrals, power
spectrum (VALU and bfloat16 MFMA), forward-mode gradient rows and the
reverse-mode adjoint, and a learned equivariant channel compression, as
hand-written HIP kernels behind a C ABI
(include/soap_mi355x.h).  This package is the thin Python binding."""
from ._lib import (SOAP_BF16_F32ACC, SOAP_F32, SOAP_F64, SoapError, EXPORTS, LIB_PATH)
from .soap import Calculator, Compressor, Neighbors, SOAPFunction, soap_power_spectrum_of_positions

__all__ = ["Calculator", "Compressor", "Neighbors", "SOAPFunction", "soap_power_spectrum_of_positions", "SoapError",
           "SOAP_F64", "SOAP_F32", "SOAP_BF16_F32ACC", "EXPORTS", "LIB_PATH"]
