"""Seeded synthetic inputs shared by the oracle and the GPU library."""
from .systems import (System, NCART, BOHR_PER_ANGSTROM, tiny_cube, chain, cluster,
                      batch_clusters, slab, config, assemble, cube_atoms,
                      sphere_atoms, chain_atoms, box_atoms, make_density)
