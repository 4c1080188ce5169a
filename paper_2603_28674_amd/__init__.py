"""Red-Green-Gray edge classification on AMD Instinct MI355X (gfx950).

``rgg`` is the binding of the C-ABI library ``librgg.so`` (HIP kernels);
``synth`` draws seeded synthetic workloads; ``build_lib`` compiles the
library in-tree.
"""
