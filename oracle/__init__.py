"""Test infrastructure: the plain CPU oracle for the PivCo-Huffman codec.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The GPU library never loads it.

The oracle itself is plain C (``pivco_ref.c``, built by ``build.py`` next to
this file); this module only marshals numpy arrays into it.
"""
from .ref import *  # noqa: F401,F403
