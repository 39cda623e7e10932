"""MI355X (gfx950) mobility product and PQN / Bi-PQN LCP solvers.

The compute path is the HIP library libbipqn.so (C ABI in include/bipqn.h);
`binding` marshals numpy arrays to it. `inputs` generates seeded workloads.
"""
