"""MI355X-native verification of Erdos' squarefree + power-of-two conjecture
on whole intervals of odd integers (Hercher, arXiv 2411.01964)."""
