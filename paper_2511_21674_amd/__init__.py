"""Event-driven e-prop on MI355X: HIP kernels behind a small C-ABI library.

``paper_2511_21674_amd.eprop`` binds the library (``libeprop_hip.so``);
``paper_2511_21674_amd.workloads`` holds the seeded synthetic inputs.
"""
