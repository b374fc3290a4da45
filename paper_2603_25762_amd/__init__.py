"""Python binding of the gfx950 haplotype-phasing library (``lib/libqhap.so``).

Argument marshalling only: torch tensors serve as device buffers and
``torch.cuda.current_stream()`` as the HIP stream; every step of the path runs
in the library's HIP kernels.  The functions mirror the C ABI in
``include/qhap.h``: :func:`build_graph` (:func:`build_graphs`), :func:`bsb_solve`,
:func:`bsb_solve_batched`, :func:`phase`, :func:`flip_crossing`, :func:`refine`.

Importing this package needs the built library and raises if it is missing;
there is no CPU fallback.
"""
from __future__ import annotations

from ._binding import (  # noqa: F401
    QhapError, Graph, build_graph, build_graphs, bsb_solve, bsb_solve_batched, phase, phase_batched,
    flip_crossing, refine,
    adaptive_schedule, autotune, load_tuned, energy_trace, refine_adaptive,
    lib_path, load, version, release_cached_memory, to_device, KIND, STORAGE, DTYPE, Status,
)
