"""MI355X-native hot path of mutual-information scan alignment
(Mehta, McBride, Pandey, arXiv 1709.06948).

The compute path is the C-ABI library ``libmi355.so`` (hand-written HIP for
gfx950) wrapped by :mod:`paper_1709_06948_amd.mi`.  :mod:`.synth` makes seeded
synthetic inputs.  Importing this package loads nothing native; importing
``.mi`` does, and fails loudly when the library is missing.
"""
__all__ = ["synth"]
