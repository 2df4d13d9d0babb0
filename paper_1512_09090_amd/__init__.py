"""MI355X-native isochrone queries (Baum, Buchhold, Dibbelt, Wagner, "Fast
Computation of Isochrones in Road Networks"): host CH preprocessing and upward
search, HIP downward sweep and isochrone-edge extraction, behind the C ABI of
include/iso.h.  This package holds the native sources (csrc/), their build
script and the ctypes binding."""
from .binding import (  # noqa: F401
    Graph, Server, Targets, IsoError, INF, TAU_MAX, MODE_PLAIN, MODE_CELLS, MODE_CD,
    ISO_OK, ISO_EINVAL, ISO_ENOMEM, ISO_EDEVICE, ISO_EFORMAT, ISO_EBUSY, ISO_ESTATE, ISO_EAGAIN, ISO_ESPACE,
    header_functions, lib,
)
