"""Fingerprint of the device sources behind the search kernel, so that stored
hardware-counter traffic is only reported while the kernel it was measured on
is unchanged."""
import hashlib
import os

_CSRC = os.path.join(os.path.dirname(os.path.abspath(__file__)), "csrc")
SEARCH_SOURCES = ("device_common.hpp", "beam.hpp", "kernels.hpp", "tiles.hpp", "mfma_score.hpp",
                  "search_impl.hpp", "search.hip", "search_mfma.hip")


def search_kernel_hash() -> str:
    h = hashlib.sha256()
    for f in SEARCH_SOURCES:
        with open(os.path.join(_CSRC, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]
