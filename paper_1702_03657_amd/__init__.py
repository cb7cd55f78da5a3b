"""MI355X (gfx950) failure-less Aho-Corasick scanner over a CRS-compressed trie.

The product is ``libpfac.so`` (HIP kernels + C ABI, see ``include/pfac.h``);
this package is its thin ctypes binding.  Importing the package does not load
the library or touch the GPU; the first call does, and fails loudly if the
library has not been built.
"""

from ._pfac import (  # noqa: F401
    MATCH_DTYPE,
    PFAC_BUILD_HOST_ONLY,
    PFAC_EBUSY,
    PFAC_EDEVICE,
    PFAC_EEMPTY,
    PFAC_EINVAL,
    PFAC_ENODEV,
    PFAC_ENOMEM,
    PFAC_ETRUNC,
    PFAC_OK,
    SIGNATURES,
    Graph,
    PfacError,
    Server,
    Trie,
    Workspace,
    load,
    matches_to_numpy,
    pfac_autotune,
    pfac_autotune_batch,
    pfac_scan,
    pfac_scan_batch,
    pfac_scan_batch_plain,
    pfac_scan_noalloc,
    pfac_scan_sync,
    scan_host,
    strerror,
)
