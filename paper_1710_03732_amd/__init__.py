"""RLT2 Lagrangian dual ascent for the QAP on one MI355X (HIP, gfx950).

``binding`` wraps the C ABI of the HIP library (include/qap_rlt2.h);
``instances`` draws the seeded synthetic workloads.  Importing the package
loads nothing; the first binding call loads the built library and raises if
it is missing.
"""
__all__ = ["binding", "instances"]
