"""MI355X (gfx950) search library for the constant-auxiliary-space heuristic of
Nag & Karforma (arXiv 1508.06561): one query, or a batch, against a protein
database, ranked, with alignments for the best hits.  The work runs in the
HIP kernels of libhs.so behind the C ABI of include/hs.h; this package is the
Python binding of that ABI."""
from .hs import (ALPHABET, Alignment, Batch, HSError, Database, DeviceSearch, Params, Result,
                 Server, align, align_batch, align_batch_dev, align_workspace_bytes, builtin_matrix,
                 encode, lib, params_default, search_batch)

__all__ = ["ALPHABET", "Alignment", "Batch", "HSError", "Database", "DeviceSearch", "Params",
           "Result", "Server", "align", "align_batch", "align_batch_dev", "align_workspace_bytes",
           "builtin_matrix", "encode", "lib", "params_default", "search_batch"]
