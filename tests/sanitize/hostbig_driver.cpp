// Test driver: the library's host big integers (hostbig.hpp) on operands read
// from stdin, one case per line "op a b m" in hexadecimal, each result printed
// in hexadecimal on its own line.  Built with AddressSanitizer and UBSan by
// the test suite, which checks the results against Python integers.
//   add a b      a + b              sub a b     a - b (a >= b)
//   mul a b      a * b              shl a s     a << s     shr a s   a >> s
//   divmod a b   "quotient remainder"           powmod a e m   a^e mod m
//   mulmod a b m (a * b) mod m      ninv a      -a^-1 mod 2^32 (a odd)
#include <stdint.h>

#include <iostream>
#include <sstream>
#include <string>

#include "../../paper_2501_07535_amd/csrc/hostbig.hpp"

using moma::HBig;

static HBig parse(const std::string& h) {
  HBig r;
  std::string d = h.substr(0, 2) == "0x" ? h.substr(2) : h;
  for (char ch : d) {
    int v = (ch >= '0' && ch <= '9') ? ch - '0' : (ch - 'a' + 10);
    r = HBig::add(HBig::shl(r, 4), HBig((uint64_t)v));
  }
  return r;
}

int main() {
  std::string line;
  while (std::getline(std::cin, line)) {
    std::istringstream in(line);
    std::string op, a, b, m;
    in >> op >> a >> b >> m;
    if (op == "add") {
      std::cout << HBig::add(parse(a), parse(b)).hex() << "\n";
    } else if (op == "sub") {
      std::cout << HBig::sub(parse(a), parse(b)).hex() << "\n";
    } else if (op == "mul") {
      std::cout << HBig::mul(parse(a), parse(b)).hex() << "\n";
    } else if (op == "shl") {
      std::cout << HBig::shl(parse(a), std::stoi(b)).hex() << "\n";
    } else if (op == "shr") {
      std::cout << HBig::shr(parse(a), std::stoi(b)).hex() << "\n";
    } else if (op == "divmod") {
      HBig q, r;
      HBig::divmod(parse(a), parse(b), &q, &r);
      std::cout << q.hex() << " " << r.hex() << "\n";
    } else if (op == "mulmod") {
      std::cout << HBig::mulmod(parse(a), parse(b), parse(m)).hex() << "\n";
    } else if (op == "powmod") {
      std::cout << HBig::powmod(parse(a), parse(b), parse(m)).hex() << "\n";
    } else if (op == "ninv") {
      uint32_t w[1];
      parse(a).to_limbs(w, 1);
      std::cout << HBig((uint64_t)moma::neg_inv32(w[0])).hex() << "\n";
    } else {
      std::cout << "?\n";
    }
  }
  return 0;
}
