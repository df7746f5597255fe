"""Batched Levenshtein / Needleman-Wunsch dynamic programs for MI355X (gfx950).

The device library is loaded lazily by ``paper_2601_15458_amd.msadp`` so that
the input generators in ``paper_2601_15458_amd.synth`` can be imported on a
machine without a GPU.
"""
