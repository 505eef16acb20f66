"""MI355X-native PivCo-Huffman: gfx950 HIP kernels behind a C ABI
(``include/pivco.h``) with a thin ctypes binding (``pivco``)."""
from .pivco import (BatchPlan, PivcoError, Tune, Workspace, lib, pivco_autotune,  # noqa: F401
                    pivco_build_tree, pivco_decode, pivco_decode_batch, pivco_decode_plain,
                    pivco_decode_workspace, pivco_encode, pivco_encode_bound,
                    pivco_merge_variants, pivco_stream_info, Server, view_output)
