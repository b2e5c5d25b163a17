"""CPU oracle for the level-blocked matrix power kernel -- TEST INFRASTRUCTURE.

Only the tests, the smoke check and the benchmark's CPU-baseline leg may use
this package.  The product library never imports it, and it imports nothing
from the product.  See ``oracle.reference`` for the functions and the paper
passages each one follows.
"""
from .reference import *  # noqa: F401,F403
